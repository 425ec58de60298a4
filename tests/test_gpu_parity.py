"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the
same seeded inputs.  Labels, moves, gains and aggregated graphs must be bit-exact;
modularity must agree to a relative 1e-9.  Run on an MI355X only."""
import zlib

import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth

pytestmark = pytest.mark.gpu

MODES = {"exact": 0, "alg1": 1, "uncond": 2, "std": 3}


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_02268_amd as m
    m.lib()
    return m


def _t(x, dev="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(dev)


def _np(t):
    return t.cpu().numpy()


def q_close(a, b):
    return abs(a - b) <= 1e-9 * max(abs(b), 1e-300) + 1e-15


GRAPHS = {
    "er200": lambda: synth.random_small(200, 0.06, 8, seed=1, loops=True),
    "er120dense": lambda: synth.random_small(120, 0.3, 8, seed=2),
    "rmat11": lambda: synth.rmat(scale=11, edge_factor=8, seed=3),
    "cl12": lambda: synth.chung_lu(n=1 << 12, avg_deg=24, seed=4),
    "planted": lambda: synth.planted_exact(n_comm=8, comm_size=60, seed=5)[0],
    "road": lambda: synth.road_like(40, seed=6),
    "kmer": lambda: synth.kmer_like(3000, seed=7),
}
_cache = {}


def graph(name):
    if name not in _cache:
        _cache[name] = GRAPHS[name]()
    return _cache[name]


# ---------------------------------------------------------------------------------
# one sweep
# ---------------------------------------------------------------------------------

@pytest.mark.parametrize("gname", ["er200", "er120dense", "rmat11", "cl12"])
@pytest.mark.parametrize("mode", ["exact", "alg1", "uncond", "std"])
# L = 1 and 2 give rows of several aligned groups of 64 chunks on the R-MAT graph
@pytest.mark.parametrize("k,L", [(1, 128), (4, 7), (8, 128), (8, 16), (16, 5), (8, 2), (4, 1),
                                 (32, 128), (64, 16), (64, 3), (32, 1), (128, 128), (128, 2),
                                 (256, 3), (256, 1)])
def test_sweep_parity(mg, gname, mode, k, L):
    g = graph(gname)
    dg = mg.to_device(g)
    rng = np.random.default_rng(zlib.crc32(f"{gname}-{mode}-{k}-{L}".encode()))
    C = rng.integers(0, max(2, g.n // 5), size=g.n).astype(np.int32)
    for algo, oalgo in ((mg.ALGO_LPA, oracle.ALGO_LPA), (mg.ALGO_LOUVAIN, oracle.ALGO_MOVE)):
        for direction in (-1, 0, 1):
            Cn, gain, ctr = mg.move_sweep(dg, algo, _t(C), direction, mode=MODES[mode], k=k,
                                          chunk_len=L)
            eC, eg = oracle.move_sweep(g, oalgo, C, mode=MODES[mode], k=k, chunk_len=L,
                                       direction=direction)
            assert np.array_equal(_np(Cn), eC), (algo, direction)
            if algo == mg.ALGO_LOUVAIN:
                assert np.array_equal(_np(gain), eg)
                assert ctr == [int((eC != C).sum()), int((eg > 0).sum()), int(eg.sum())]
            else:
                assert ctr[0] == int((eC != C).sum())


@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12"])
@pytest.mark.parametrize("mode,k,L", [("exact", 8, 128), ("alg1", 2, 9), ("alg1", 16, 128),
                                      ("std", 4, 6), ("alg1", 64, 128), ("std", 32, 7),
                                      ("uncond", 64, 20), ("alg1", 128, 3), ("std", 256, 1),
                                      ("uncond", 128, 64)])
def test_refine_parity(mg, gname, mode, k, L):
    g = graph(gname)
    dg = mg.to_device(g)
    rng = np.random.default_rng(11)
    bound = rng.integers(0, max(2, g.n // 40), size=g.n).astype(np.int32)
    R = mg.refine(dg, _t(bound), mode=MODES[mode], k=k, chunk_len=L)
    eR = oracle.refine(g, bound, mode=MODES[mode], k=k, chunk_len=L)
    assert np.array_equal(_np(R), eR)


@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12", "planted"])
@pytest.mark.parametrize("mode,k,L", [("exact", 8, 128), ("alg1", 1, 128), ("alg1", 4, 11),
                                      ("alg1", 8, 128), ("alg1", 16, 40), ("uncond", 8, 64),
                                      ("alg1", 64, 128), ("alg1", 32, 5), ("std", 64, 9),
                                      ("uncond", 32, 64), ("alg1", 8, 1), ("std", 4, 2),
                                      ("alg1", 128, 128), ("alg1", 256, 2), ("std", 128, 9),
                                      ("uncond", 256, 4)])
@pytest.mark.parametrize("symmetric", [False, True])
def test_aggregate_parity(mg, gname, mode, k, L, symmetric):
    g = graph(gname)
    dg = mg.to_device(g)
    rng = np.random.default_rng(5)
    C = rng.integers(0, max(2, g.n // 7), size=g.n)
    u, D = np.unique(C, return_inverse=True)
    m = len(u)
    off, idx, w = mg.aggregate(dg, _t(D), m, symmetric, mode=MODES[mode], k=k, chunk_len=L)
    e = oracle.aggregate(g, D.astype(np.int32), m, mode=MODES[mode], k=k, chunk_len=L,
                         symmetric=symmetric)
    assert np.array_equal(off, e.offsets)
    assert np.array_equal(idx, e.indices)
    assert np.array_equal(w, e.weights)


# ---------------------------------------------------------------------------------
# whole runs
# ---------------------------------------------------------------------------------

RUNS = [
    ("lpa", "exact", 8, 128), ("lpa", "alg1", 8, 128), ("lpa", "alg1", 2, 6), ("lpa", "std", 4, 128),
    ("louvain", "exact", 8, 128), ("louvain", "alg1", 8, 128), ("louvain", "alg1", 16, 9),
    ("louvain", "uncond", 4, 128), ("louvain", "std", 8, 32), ("louvain", "alg1", 1, 128),
    ("leiden", "exact", 16, 128), ("leiden", "alg1", 16, 128), ("leiden", "alg1", 8, 10),
    ("leiden", "std", 4, 128),
    ("leiden", "alg1", 64, 128), ("louvain", "alg1", 32, 16), ("lpa", "alg1", 64, 5),
    ("leiden", "uncond", 32, 128), ("louvain", "std", 64, 128),
    ("leiden", "alg1", 128, 128), ("louvain", "alg1", 256, 16), ("lpa", "std", 128, 5),
    ("louvain", "uncond", 256, 128), ("leiden", "alg1", 256, 3),
]


@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12", "planted", "road", "kmer"])
@pytest.mark.parametrize("algo,mode,k,L", RUNS)
def test_run_parity(mg, gname, algo, mode, k, L):
    g = graph(gname)
    dg = mg.to_device(g)
    kw = dict(mode=MODES[mode], k=k, chunk_len=L)
    lab, st = getattr(mg, algo)(dg, **kw)
    elab, est = getattr(oracle, algo)(g, **kw)
    lab = _np(lab)
    assert np.array_equal(lab, elab)
    assert st["iterations"] == est.iterations and st["passes"] == est.passes
    assert st["communities"] == est.communities
    assert st["edges_scanned"] == est.edges_scanned
    q = mg.modularity(dg, _t(lab))
    assert q_close(q, oracle.modularity(g, elab))


def test_edge_cases(mg):
    import torch
    # isolated vertices, a self-loop only vertex, one edge
    g = synth.from_edges(6, [(0, 1)], self_loops={4: 3})
    dg = mg.to_device(g)
    for algo in ("lpa", "louvain", "leiden"):
        for mode in (0, 1):
            lab, st = getattr(mg, algo)(dg, mode=mode, k=4)
            elab, est = getattr(oracle, algo)(g, mode=mode, k=4)
            assert np.array_equal(_np(lab), elab)
    # K2 oscillates under synchronous LPA until the sweep cap
    k2 = mg.to_device(synth.from_edges(2, [(0, 1)]))
    lab, st = mg.lpa(k2, mode=0)
    assert st["iterations"] == 20 and list(_np(lab)) == [0, 1]
    # one vertex without edges
    one = mg.to_device(synth.from_edges(1, []))
    lab, st = mg.louvain(one)
    assert list(_np(lab)) == [0]
    # total weight at 2^31 is rejected
    big = synth.from_edges(2, [(0, 1)], weights=[1 << 30])
    with pytest.raises(mg.MgcdError) as ei:
        mg.louvain(mg.to_device(big))
    assert ei.value.code == -3
    # validation catches an index out of range
    bad = synth.from_edges(3, [(0, 1), (1, 2)])
    bad.indices = bad.indices.copy()
    bad.indices[0] = 7
    with pytest.raises(mg.MgcdError) as ei:
        mg.lpa(mg.to_device(bad), validate=1)
    assert ei.value.code == -2
    # unsupported k
    with pytest.raises(mg.MgcdError) as ei:
        mg.louvain(mg.to_device(synth.from_edges(3, [(0, 1)])), k=3)
    assert ei.value.code == -6
    # labels out of range are rejected before any indexing
    with pytest.raises(mg.MgcdError):
        mg.modularity(dg, torch.full((6,), 9, dtype=torch.int32, device="cuda"))


def test_workspace_too_small(mg):
    import ctypes as ct
    import torch
    g = mg.to_device(synth.random_small(50, 0.1, 3, seed=9))
    p = mg.params(mg.ALGO_LOUVAIN)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    d = g.desc()
    rc = mg.lib().louvain_run(ct.byref(d), ct.byref(p), out.data_ptr(), ws.data_ptr(), 1024, None,
                              mg._stream())
    assert rc == -4


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("labels", ["50", "one", "giant", "distinct"])
def test_modularity_parity(mg, seed, labels):
    """Q against the oracle for 50 random communities, a single community, one giant
    community (90 % of the vertices) among singletons, and all vertices apart (the
    per-workgroup combining of community totals: one key, few keys, all distinct)."""
    g = synth.rmat(scale=12, edge_factor=8, seed=20 + seed)
    rng = np.random.default_rng(seed)
    if labels == "50":
        C = rng.integers(0, 50, size=g.n)
    elif labels == "one":
        C = np.zeros(g.n)
    elif labels == "giant":
        C = np.where(rng.random(g.n) < 0.9, 7, np.arange(g.n))
    else:
        C = rng.permutation(g.n)
    C = C.astype(np.int32)
    q = mg.modularity(mg.to_device(g), _t(C))
    assert q_close(q, oracle.modularity(g, C))


# ---------------------------------------------------------------------------------
# the configured workloads
# ---------------------------------------------------------------------------------

def test_planted_lpa_config(mg):
    """LPA, MG k=8, planted partition 20 x 500, 12 intra + 4 inter edges, <= 20 sweeps."""
    g, truth = synth.planted_exact()
    dg = mg.to_device(g)
    for mode in (1, 0):
        lab, st = mg.lpa(dg, mode=mode, k=8)
        elab, est = oracle.lpa(g, mode=mode, k=8)
        assert np.array_equal(_np(lab), elab)
        assert st["iterations"] == est.iterations <= 20


@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12", "road", "kmer"])
@pytest.mark.parametrize("algo,mode,k,L", [("lpa", "alg1", 8, 128), ("louvain", "alg1", 1, 128),
                                           ("louvain", "std", 4, 2), ("leiden", "alg1", 16, 128),
                                           ("leiden", "std", 8, 5), ("louvain", "uncond", 4, 128)])
def test_short_rows_schedule_only(mg, gname, algo, mode, k, L):
    """Rows of at most k entries on the exact one-lane kernel (short_rows = 2), on the
    sketch kernels (1) or by the graph's average row (0): the same labels and counts,
    equal to the oracle's."""
    g = graph(gname)
    dg = mg.to_device(g)
    kw = dict(mode=MODES[mode], k=k, chunk_len=L)
    elab, est = getattr(oracle, algo)(g, **kw)
    runs = [getattr(mg, algo)(dg, short_rows=sr, **kw) for sr in (0, 1, 2)]
    for lab, st in runs:
        assert np.array_equal(_np(lab), elab)
        for key in ("iterations", "passes", "edges_scanned", "moved_last"):
            assert st[key] == runs[0][1][key]


@pytest.mark.parametrize("cls", ["road", "kmer"])
@pytest.mark.parametrize("algo,mode,k", [("lpa", "alg1", 8), ("louvain", "alg1", 8), ("leiden", "alg1", 16),
                                         ("louvain", "exact", 8), ("lpa", "exact", 8)])
def test_low_degree_class_config(mg, cls, algo, mode, k):
    """The road and k-mer stand-ins at a million vertices (about 2.1 entries per
    vertex): whole runs equal the oracle's labels and counts."""
    key = cls + "_big"
    if key not in _cache:
        _cache[key] = (synth.road_like(480, seed=4, device="cuda") if cls == "road"
                       else synth.kmer_like(1 << 20, seed=5, device="cuda"))
    g = _cache[key]
    dg = mg.to_device(g)
    kw = dict(mode=MODES[mode], k=k, chunk_len=128)
    lab, st = getattr(mg, algo)(dg, **kw)
    elab, est = getattr(oracle, algo)(g, **kw)
    assert np.array_equal(_np(lab), elab)
    assert st["iterations"] == est.iterations and st["passes"] == est.passes
    assert st["edges_scanned"] == est.edges_scanned


def test_rmat20_louvain_config(mg):
    """Louvain MG k=8 on the R-MAT 2^20 graph (~31M CSR entries), the benchmarked
    workload: labels bit-exact with the oracle."""
    g = synth.rmat()
    dg = mg.to_device(g)
    lab, st = mg.louvain(dg, mode=1, k=8)
    elab, est = oracle.louvain(g, mode=1, k=8)
    assert np.array_equal(_np(lab), elab)
    assert st["iterations"] == est.iterations and st["passes"] == est.passes
    assert q_close(mg.modularity(dg, lab), oracle.modularity(g, elab))
    # exact mode: one full-size sweep against the oracle (the full exact run is slow on CPU)
    C = np.arange(g.n, dtype=np.int32)
    Cn, gain, ctr = mg.move_sweep(dg, mg.ALGO_LOUVAIN, _t(C), -1, mode=0)
    eC, eg = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=0, direction=-1)
    assert np.array_equal(_np(Cn), eC) and np.array_equal(_np(gain), eg)


# ---------------------------------------------------------------------------------
# batched runs
# ---------------------------------------------------------------------------------

def _batch_graphs():
    gs = []
    rng = np.random.default_rng(77)
    for q in range(14):
        n = int(rng.integers(60, 1500))
        gs.append(synth.planted_uneven(n, 20, 200, 6, 4, rng)[0])
    gs.append(synth.rmat(scale=10, edge_factor=8, seed=78))
    gs.append(synth.from_edges(5, []))            # isolated vertices only
    gs.append(synth.from_edges(0, []))            # empty graph
    gs.append(synth.chung_lu(n=1 << 11, avg_deg=20, seed=79))
    gs.append(synth.from_edges(2, [(0, 1)]))      # K2
    return gs


@pytest.mark.parametrize("algo", ["lpa", "louvain"])
@pytest.mark.parametrize("mode,k,L,direct", [("alg1", 8, 128, 0), ("alg1", 4, 16, 0),
                                             ("exact", 8, 128, 0), ("alg1", 32, 16, 0),
                                             ("alg1", 64, 128, 0), ("alg1", 8, 128, 1),
                                             ("exact", 8, 128, 1)])
def test_batched_equals_solo(mg, algo, mode, k, L, direct):
    gs = _batch_graphs()
    dgs = [mg.to_device(g) for g in gs]
    kw = dict(mode=MODES[mode], k=k, chunk_len=L)
    code = mg.ALGO_LPA if algo == "lpa" else mg.ALGO_LOUVAIN
    labs, gst, tot = mg.run_batched(code, dgs, direct_launch=direct, **kw)
    again, _, _ = mg.run_batched(code, dgs, direct_launch=direct, **kw)  # a second call agrees
    for x, y in zip(labs, again):
        assert np.array_equal(_np(x), _np(y))
    for g, dg, lab, st in zip(gs, dgs, labs, gst):
        if g.n == 0:
            assert lab.numel() == 0
            continue
        solo, sst = getattr(mg, algo)(dg, **kw)
        assert np.array_equal(_np(lab), _np(solo))
        assert st["iterations"] == sst["iterations"] and st["passes"] == sst["passes"]
        assert st["communities"] == sst["communities"]
        assert st["edges_scanned"] == sst["edges_scanned"]
        elab, est = getattr(oracle, algo)(g, **kw)
        assert np.array_equal(_np(lab), elab)


@pytest.mark.parametrize("k", [8, 16, 32, 64, 128, 256])
def test_wave_sketch_deep_merge_tree(mg, k):
    """A hub row of 6,000 entries with L = 1: a merge tree of more than 4,096 chunk
    sketches (the deep stack of the wave sketch at k >= 32; about 94 groups of 64
    chunks at k <= 16); its sweep and aggregation match the oracle."""
    rng = np.random.default_rng(31)
    n = 6001
    edges = [(0, v) for v in range(1, n)]
    edges += [(int(u), int(v)) for u, v in rng.integers(1, n, size=(3000, 2)) if u != v]
    w = rng.integers(1, 9, size=len(edges)).astype(np.uint32)
    g = synth.from_edges(n, edges, w)
    dg = mg.to_device(g)
    C = rng.integers(0, 300, size=n).astype(np.int32)
    for algo, oalgo in ((mg.ALGO_LPA, oracle.ALGO_LPA), (mg.ALGO_LOUVAIN, oracle.ALGO_MOVE)):
        Cn, gain, _ = mg.move_sweep(dg, algo, _t(C), 0, mode=mg.MODE_ALG1, k=k, chunk_len=1)
        eC, eg = oracle.move_sweep(g, oalgo, C, mode=oracle.MODE_ALG1, k=k, chunk_len=1)
        assert np.array_equal(_np(Cn), eC)
    u, D = np.unique(rng.integers(0, 40, size=n), return_inverse=True)
    off, idx, ww = mg.aggregate(dg, _t(D), len(u), False, mode=mg.MODE_ALG1, k=k, chunk_len=1)
    e = oracle.aggregate(g, D.astype(np.int32), len(u), mode=oracle.MODE_ALG1, k=k, chunk_len=1)
    assert np.array_equal(off, e.offsets) and np.array_equal(idx, e.indices)
    assert np.array_equal(ww, e.weights)


# exact_small / exact_lds / exact_lds_big of (2, 8, 24) put rows on every table tier
# (registers, row-sized and 8,192-slot LDS tables, global tables)
TIERS = {"default": {}, "all_tiers": dict(exact_small=2, exact_lds=8, exact_lds_big=24)}


def _hub_graph(seed):
    """6,000 vertices; five hubs of 5,000, 2,049, 1,300, 701 and 513 random neighbours
    (chunk counts that are not powers of two) plus 8,000 random edges, weights 1..8."""
    rng = np.random.default_rng(seed)
    n = 6000
    edges = []
    for h, deg in enumerate((5000, 2049, 1300, 701, 513)):
        edges += [(h, int(v)) for v in rng.choice(np.arange(5, n), size=deg, replace=False)]
    edges += [(int(u), int(v)) for u, v in rng.integers(5, n, size=(8000, 2)) if u != v]
    w = rng.integers(1, 9, size=len(edges)).astype(np.uint32)
    return synth.from_edges(n, edges, w)


@pytest.mark.parametrize("k", [32, 64, 128, 256])
@pytest.mark.parametrize("mode", ["alg1", "uncond", "std"])
@pytest.mark.parametrize("L", [1, 37, 128, 700])
def test_wave_split_rows(mg, k, mode, L):
    """At k = 32/64, rows of more than max(L, 512) entries are sketched one wave per
    chunk and merged level by level on the device: labels, gains and counters equal the
    oracle's for LPA, Louvain, 1-scan LPA and the refinement sweep, with neighbour
    labels from 20 communities (loss-free hub sketches) and from 3,000 (lossy); the
    aggregation of streams longer than max(L, 512) positions likewise."""
    g = _hub_graph(77)
    dg = mg.to_device(g)
    rng = np.random.default_rng(zlib.crc32(f"split-{k}-{mode}-{L}".encode()))
    for ncomm in (20, 3000):
        C = rng.integers(0, ncomm, size=g.n).astype(np.int32)
        for algo, oalgo in ((mg.ALGO_LPA, oracle.ALGO_LPA), (mg.ALGO_LOUVAIN, oracle.ALGO_MOVE)):
            Cn, gain, ctr = mg.move_sweep(dg, algo, _t(C), 0, mode=MODES[mode], k=k, chunk_len=L)
            eC, eg = oracle.move_sweep(g, oalgo, C, mode=MODES[mode], k=k, chunk_len=L)
            assert np.array_equal(_np(Cn), eC), (algo, ncomm)
            if algo == mg.ALGO_LOUVAIN:
                assert np.array_equal(_np(gain), eg)
                assert ctr == [int((eC != C).sum()), int((eg > 0).sum()), int(eg.sum())]
        Cn, _, _ = mg.move_sweep(dg, mg.ALGO_LPA, _t(C), 0, mode=MODES[mode], k=k, chunk_len=L,
                                 one_scan=1)
        eC, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=MODES[mode], k=k, chunk_len=L,
                                  one_scan=1)
        assert np.array_equal(_np(Cn), eC), ("1-scan", ncomm)
    bound = rng.integers(0, 3, size=g.n).astype(np.int32)
    R = mg.refine(dg, _t(bound), mode=MODES[mode], k=k, chunk_len=L)
    eR = oracle.refine(g, bound, mode=MODES[mode], k=k, chunk_len=L)
    assert np.array_equal(_np(R), eR)
    # aggregation: community streams longer than max(L, 512) positions are split the same way
    for ncomm in (5, 300):
        u, D = np.unique(rng.integers(0, ncomm, size=g.n), return_inverse=True)
        for symmetric in (False, True):
            off, idx, ww = mg.aggregate(dg, _t(D), len(u), symmetric, mode=MODES[mode], k=k,
                                        chunk_len=L)
            e = oracle.aggregate(g, D.astype(np.int32), len(u), mode=MODES[mode], k=k,
                                 chunk_len=L, symmetric=symmetric)
            assert np.array_equal(off, e.offsets), (ncomm, symmetric)
            assert np.array_equal(idx, e.indices) and np.array_equal(ww, e.weights)


@pytest.mark.parametrize("mode,k", [("exact", 8), ("small", 3), ("small", 4096)])
@pytest.mark.parametrize("tiers", sorted(TIERS))
def test_exact_segmented_rows(mg, mode, k, tiers):
    """Exact and small-table modes with rows of more than 4,096 entries: a row's global
    table filled by several workgroups (segments of 4,096 entries) and decided by one.
    Sweeps, the refinement sweep and whole Louvain, Leiden and LPA runs (a level's
    sweeps reuse the tables, which each decision clears) equal the oracle's."""
    g = _hub_graph(78)
    dg = mg.to_device(g)
    gm = mg.MODE_EXACT if mode == "exact" else mg.MODE_SMALL
    om = oracle.MODE_EXACT if mode == "exact" else oracle.MODE_SMALL
    rng = np.random.default_rng(zlib.crc32(f"gseg-{mode}-{k}-{tiers}".encode()))
    for ncomm in (20, 3000):
        C = rng.integers(0, ncomm, size=g.n).astype(np.int32)
        for algo, oalgo in ((mg.ALGO_LPA, oracle.ALGO_LPA), (mg.ALGO_LOUVAIN, oracle.ALGO_MOVE)):
            Cn, gain, ctr = mg.move_sweep(dg, algo, _t(C), 0, mode=gm, k=k, **TIERS[tiers])
            eC, eg = oracle.move_sweep(g, oalgo, C, mode=om, k=k)
            assert np.array_equal(_np(Cn), eC), (algo, ncomm)
            if algo == mg.ALGO_LOUVAIN:
                assert np.array_equal(_np(gain), eg)
                assert ctr == [int((eC != C).sum()), int((eg > 0).sum()), int(eg.sum())]
    bound = rng.integers(0, 3, size=g.n).astype(np.int32)
    R = mg.refine(dg, _t(bound), mode=gm, k=k, **TIERS[tiers])
    assert np.array_equal(_np(R), oracle.refine(g, bound, mode=om, k=k))
    for algo in ("louvain", "leiden", "lpa"):
        lab, st = getattr(mg, algo)(dg, mode=gm, k=k, **TIERS[tiers])
        elab, est = getattr(oracle, algo)(g, mode=om, k=k)
        assert np.array_equal(_np(lab), elab), algo
        assert st["iterations"] == est.iterations


@pytest.mark.parametrize("gname", ["er120dense", "rmat11"])
@pytest.mark.parametrize("mode,k", [("exact", 8), ("small", 5)])
def test_exact_every_row_on_global_tables(mg, gname, mode, k):
    """Tier thresholds of 1 put every row of two or more entries on a global table (as
    many table rows as vertices): the workspace the library reports suffices, and
    sweeps and whole runs equal the oracle's."""
    g = graph(gname)
    dg = mg.to_device(g)
    gm = mg.MODE_EXACT if mode == "exact" else mg.MODE_SMALL
    om = oracle.MODE_EXACT if mode == "exact" else oracle.MODE_SMALL
    kw = dict(exact_small=1, exact_lds=1, exact_lds_big=1)
    C = np.random.default_rng(3).integers(0, max(2, g.n // 4), size=g.n).astype(np.int32)
    Cn, gain, _ = mg.move_sweep(dg, mg.ALGO_LOUVAIN, _t(C), 0, mode=gm, k=k, **kw)
    eC, eg = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=om, k=k)
    assert np.array_equal(_np(Cn), eC) and np.array_equal(_np(gain), eg)
    for algo in ("louvain", "leiden", "lpa"):
        lab, _ = getattr(mg, algo)(dg, mode=gm, k=k, **kw)
        elab, _ = getattr(oracle, algo)(g, mode=om, k=k)
        assert np.array_equal(_np(lab), elab), algo


@pytest.mark.parametrize("algo", ["lpa", "louvain"])
@pytest.mark.parametrize("mode,k,L", [("alg1", 64, 128), ("alg1", 32, 37), ("std", 64, 1),
                                      ("exact", 8, 128)])
def test_batched_with_hub_rows(mg, algo, mode, k, L):
    """Batched runs where two graphs have hub rows of 513 to 5,000 entries (split rows of
    the 32/64-slot sketch, segmented global tables of the exact mode) next to small
    graphs that converge first, so the hub graphs' long rows are swept while other
    graphs are frozen and vice versa: every graph equals its plain run and the oracle."""
    gs = _batch_graphs() + [_hub_graph(90), _hub_graph(91)]
    dgs = [mg.to_device(g) for g in gs]
    kw = dict(mode=MODES[mode], k=k, chunk_len=L)
    code = mg.ALGO_LPA if algo == "lpa" else mg.ALGO_LOUVAIN
    labs, gst, _ = mg.run_batched(code, dgs, **kw)
    for g, dg, lab, st in zip(gs, dgs, labs, gst):
        if g.n == 0:
            continue
        solo, sst = getattr(mg, algo)(dg, **kw)
        assert np.array_equal(_np(lab), _np(solo))
        assert st["iterations"] == sst["iterations"] and st["edges_scanned"] == sst["edges_scanned"]
        elab, _ = getattr(oracle, algo)(g, **kw)
        assert np.array_equal(_np(lab), elab)


@pytest.mark.parametrize("algo", ["lpa", "louvain"])
def test_batched_many_graphs_dirty_workspace(mg, algo):
    """More graphs than one wave of counters, in a workspace full of garbage: every
    per-graph counter and statistic must start from zero (regression: a clear that
    covered only 64 entries)."""
    import torch
    gs = [synth.planted_uneven(n, 20, 200, 6, 4, np.random.default_rng(900 + n))[0]
          for n in range(300, 300 + 45 * 37, 37)]
    dgs = [mg.to_device(g) for g in gs]
    code = mg.ALGO_LPA if algo == "lpa" else mg.ALGO_LOUVAIN
    kw = dict(mode=mg.MODE_ALG1, k=8, chunk_len=16)
    nbytes = mg.batched_workspace_bytes(code, dgs, **kw)
    ws = torch.full((nbytes,), 0xA7, dtype=torch.uint8, device="cuda")
    labs, gst, tot = mg.run_batched(code, dgs, workspace=ws, **kw)
    for dg, lab, st in zip(dgs, labs, gst):
        solo, sst = getattr(mg, algo)(dg, **kw)
        assert np.array_equal(_np(lab), _np(solo))
        for key in ("iterations", "passes", "communities", "edges_scanned", "moved_last"):
            assert st[key] == sst[key], key


# ---------------------------------------------------------------------------------
# LPA, the 1-scan variant (Section 4.3): decisions from the sketch's values
# ---------------------------------------------------------------------------------

@pytest.mark.gpu
@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12"])
@pytest.mark.parametrize("mode", ["alg1", "uncond", "std"])
# L = 1 and 2 put the R-MAT hubs on the long-row path; k = 32 and 64 use the wave sketch
@pytest.mark.parametrize("k,L", [(1, 128), (4, 7), (8, 2), (16, 5), (8, 1), (32, 128), (64, 16)])
def test_lpa_one_scan_sweep_parity(mg, gname, mode, k, L):
    g = graph(gname)
    dg = mg.to_device(g)
    rng = np.random.default_rng(zlib.crc32(f"1scan-{gname}-{mode}-{k}-{L}".encode()))
    C = rng.integers(0, max(2, g.n // 5), size=g.n).astype(np.int32)
    Cn, _, ctr = mg.move_sweep(dg, mg.ALGO_LPA, _t(C), 0, mode=MODES[mode], k=k, chunk_len=L,
                               one_scan=1)
    eC, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=MODES[mode], k=k, chunk_len=L,
                              one_scan=1)
    assert np.array_equal(_np(Cn), eC)
    assert ctr[0] == int((eC != C).sum())


@pytest.mark.gpu
@pytest.mark.parametrize("k,L", [(1, 128), (8, 128), (8, 4), (64, 16)])
def test_lpa_one_scan_run_parity(mg, k, L):
    for gname in ("rmat11", "planted", "cl12"):
        g = graph(gname)
        dg = mg.to_device(g)
        lab, st = mg.lpa(dg, k=k, chunk_len=L, one_scan=1)
        elab, est = oracle.lpa(g, k=k, chunk_len=L, one_scan=1)
        assert np.array_equal(_np(lab), elab), gname
        assert st["iterations"] == est.iterations and st["edges_scanned"] == est.edges_scanned
    # batched runs take the same decisions
    gs = _batch_graphs()
    dgs = [mg.to_device(g) for g in gs]
    labs, gst, _ = mg.run_batched(mg.ALGO_LPA, dgs, k=k, chunk_len=L, one_scan=1)
    for g, lab in zip(gs, labs):
        if g.n:
            elab, _ = oracle.lpa(g, k=k, chunk_len=L, one_scan=1)
            assert np.array_equal(_np(lab), elab)


@pytest.mark.gpu
def test_one_scan_is_lpa_only(mg):
    dg = mg.to_device(graph("er200"))
    for fn in (mg.louvain, mg.leiden):
        with pytest.raises(mg.MgcdError) as ei:
            fn(dg, one_scan=1)
        assert ei.value.code == -6
    with pytest.raises(mg.MgcdError) as ei:
        mg.run_batched(mg.ALGO_LOUVAIN, [dg], one_scan=1)
    assert ei.value.code == -6
    with pytest.raises(mg.MgcdError) as ei:
        mg.lpa(dg, one_scan=2)
    assert ei.value.code == -1


@pytest.mark.gpu
def test_boyer_moore_mode(mg):
    # MGCD_MODE_BM resolves to Algorithm 1 with k = 1 (moving, refinement) and
    # k_aggregate = 4, on the device and in the oracle alike
    for gname in ("rmat11", "planted"):
        g = graph(gname)
        dg = mg.to_device(g)
        for algo in ("lpa", "louvain", "leiden"):
            lab, st = getattr(mg, algo)(dg, mode=mg.MODE_BM, k=16, chunk_len=32)
            same, sst = getattr(mg, algo)(dg, mode=mg.MODE_ALG1, k=1, k_aggregate=4, chunk_len=32)
            elab, est = getattr(oracle, algo)(g, mode=oracle.MODE_BM, chunk_len=32)
            assert np.array_equal(_np(lab), _np(same)) and np.array_equal(_np(lab), elab)
            assert st["iterations"] == est.iterations and st["passes"] == est.passes


# ---------------------------------------------------------------------------------
# the small mod-based table (Appendix A.2)
# ---------------------------------------------------------------------------------


@pytest.mark.gpu
@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12"])
@pytest.mark.parametrize("slots", [1, 3, 37, 1000, 1 << 20])
@pytest.mark.parametrize("tiers", sorted(TIERS))
def test_small_table_sweep_parity(mg, gname, slots, tiers):
    g = graph(gname)
    dg = mg.to_device(g)
    rng = np.random.default_rng(zlib.crc32(f"small-{gname}-{slots}".encode()))
    C = rng.integers(0, max(2, g.n // 5), size=g.n).astype(np.int32)
    for algo, oalgo in ((mg.ALGO_LPA, oracle.ALGO_LPA), (mg.ALGO_LOUVAIN, oracle.ALGO_MOVE)):
        Cn, gain, ctr = mg.move_sweep(dg, algo, _t(C), -1, mode=mg.MODE_SMALL, k=slots,
                                      **TIERS[tiers])
        eC, eg = oracle.move_sweep(g, oalgo, C, mode=oracle.MODE_SMALL, k=slots, direction=-1)
        assert np.array_equal(_np(Cn), eC), algo
        if algo == mg.ALGO_LOUVAIN:
            assert np.array_equal(_np(gain), eg)
    bound = rng.integers(0, 4, size=g.n).astype(np.int32)
    R = mg.refine(dg, _t(bound), mode=mg.MODE_SMALL, k=slots, **TIERS[tiers])
    eR = oracle.refine(g, bound, mode=oracle.MODE_SMALL, k=slots)
    assert np.array_equal(_np(R), eR)


@pytest.mark.gpu
@pytest.mark.parametrize("slots", [2, 50, 1 << 16])
def test_small_table_run_parity(mg, slots):
    for gname in ("planted", "rmat11"):
        g = graph(gname)
        dg = mg.to_device(g)
        for algo in ("lpa", "louvain", "leiden"):
            lab, st = getattr(mg, algo)(dg, mode=mg.MODE_SMALL, k=slots)
            elab, est = getattr(oracle, algo)(g, mode=oracle.MODE_SMALL, k=slots)
            assert np.array_equal(_np(lab), elab), (gname, algo)
            assert st["iterations"] == est.iterations and st["passes"] == est.passes
    gs = _batch_graphs()
    dgs = [mg.to_device(g) for g in gs]
    for code, algo in ((mg.ALGO_LPA, "lpa"), (mg.ALGO_LOUVAIN, "louvain")):
        labs, _, _ = mg.run_batched(code, dgs, mode=mg.MODE_SMALL, k=slots)
        for g, lab in zip(gs, labs):
            if g.n:
                elab, _ = getattr(oracle, algo)(g, mode=oracle.MODE_SMALL, k=slots)
                assert np.array_equal(_np(lab), elab)


@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12"])
@pytest.mark.parametrize("algo", ["louvain", "leiden"])
@pytest.mark.parametrize("cfg", [dict(mode=1, k=4, aggregation=1),
                                 dict(mode=0, k_aggregate=4, aggregation=2),
                                 dict(mode=1, k=32, k_aggregate=2, aggregation=2, chunk_len=37)],
                         ids=["mg-move-exact-agg", "exact-move-mg-agg", "k32-move-k2-agg"])
def test_decoupled_aggregation(mg, gname, algo, cfg):
    """Aggregation decoupled from local moving (the measurement of each phase's share
    of a sketch's modularity loss): whole runs equal to the oracle."""
    g = graph(gname)
    lab, st = getattr(mg, algo)(mg.to_device(g), **cfg)
    elab, est = getattr(oracle, algo)(g, **cfg)
    assert np.array_equal(_np(lab), elab)
    assert st["iterations"] == est.iterations and st["passes"] == est.passes


@pytest.mark.parametrize("gname", ["er200", "rmat11", "cl12", "planted"])
@pytest.mark.parametrize("algo", ["lpa", "louvain", "leiden"])
@pytest.mark.parametrize("cfg", [dict(mode=1, k=8), dict(mode=1, k=2, chunk_len=5),
                                 dict(mode=0), dict(mode=1, k=64, chunk_len=37),
                                 dict(mode=5, k=7), dict(mode=3, k=16, chunk_len=3)],
                         ids=["alg1-k8", "alg1-k2-L5", "exact", "alg1-k64-L37", "small-7", "std-k16-L3"])
def test_storage_order_changes_nothing(mg, gname, algo, cfg):
    """Level 0 on the degree-ordered storage copy (forced on): labels and counters equal
    to the oracle's (and so to the input-order run's)."""
    g = graph(gname)
    lab, st = getattr(mg, algo)(mg.to_device(g), storage_order=2, **cfg)
    elab, est = getattr(oracle, algo)(g, **cfg)
    assert np.array_equal(_np(lab), elab)
    assert st["iterations"] == est.iterations and st["passes"] == est.passes


def test_storage_order_on_rmat16(mg):
    """A larger power-law graph with isolated vertices and hub rows on the long-row
    path: the storage copy gives the input order's labels and statistics."""
    g = synth.rmat(scale=16, edge_factor=16, seed=44)
    dg = mg.to_device(g)
    for algo in ("lpa", "louvain", "leiden"):
        a, sa = getattr(mg, algo)(dg, storage_order=2)
        b, sb = getattr(mg, algo)(dg, storage_order=1)
        assert bool((a == b).all())
        for key in ("iterations", "passes", "communities", "edges_scanned", "l0_candidates"):
            assert sa[key] == sb[key], key
    elab, _ = oracle.louvain(g)
    assert np.array_equal(_np(mg.louvain(dg, storage_order=2)[0]), elab)
