"""Serving (continuous batching), by whole calls and by steps: every request's result
equals the same call made alone, whatever else is resident; admission respects the
arena; errors surface."""
import time

import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_02268_amd as m
    m.lib()
    return m


def _pool():
    gs = [synth.rmat(scale=s, edge_factor=8, seed=50 + s) for s in (9, 10, 11, 12, 13)]
    gs.append(synth.planted_exact(n_comm=6, comm_size=50, seed=7)[0])
    gs.append(synth.random_small(300, 0.05, 8, seed=8, loops=True))
    gs.append(synth.from_edges(1, []))
    return gs


@pytest.fixture(scope="module")
def pool(mg):
    return [mg.to_device(g) for g in _pool()]


def _solo(mg, algo, dg, kw):
    fn = {mg.ALGO_LPA: mg.lpa, mg.ALGO_LOUVAIN: mg.louvain, mg.ALGO_LEIDEN: mg.leiden}[algo]
    lab, st = fn(dg, **kw)
    return lab.cpu().numpy(), st


ALGOS = ["louvain", "lpa", "leiden"]


def _algo(mg, name):
    return {"lpa": mg.ALGO_LPA, "louvain": mg.ALGO_LOUVAIN, "leiden": mg.ALGO_LEIDEN}[name]


def _check_same(mg, algo, pool, server, order, kw, stepped=False):
    solo = [_solo(mg, algo, dg, kw) for dg in pool]
    tickets = [(server.submit(pool[i]), i) for i in order]
    for t, i in tickets:
        lab, st, tm = server.wait(t)
        np.testing.assert_array_equal(lab.cpu().numpy(), solo[i][0])
        keys = ["iterations", "passes", "communities", "edges_scanned"]
        if stepped:
            keys.append("moved_last")
        for key in keys:
            assert st[key] == solo[i][1][key], key
        assert tm[0] <= tm[1] <= tm[2]


@pytest.mark.parametrize("stepped", [False, True], ids=["calls", "steps"])
@pytest.mark.parametrize("algo_name", ALGOS)
def test_alone_equals_mixed(mg, pool, algo_name, stepped):
    algo = _algo(mg, algo_name)
    kw = {}
    order = [4, 0, 5, 3, 1, 7, 2, 6, 4, 4, 0]
    with mg.Server(algo, 1 << 30, slots=4, stepped=stepped, **kw) as srv:
        _check_same(mg, algo, pool, srv, order, kw, stepped)
        info = srv.info()
        assert info["waiting"] == 0 and info["running"] == 0 and info["bytes_in_use"] == 0


STEPPED_PARAMS = [
    dict(),
    dict(mode=0),                      # exact tables
    dict(k=32, k_aggregate=8),         # wave sketch, decoupled aggregation
    dict(k=4, mode=2, chunk_len=16),   # unconditional subtraction, short chunks
    dict(mode=5, k=7),                 # the small mod-based table
    dict(aggregation=1, max_iterations=3, max_passes=2),
]


@pytest.mark.parametrize("kw", STEPPED_PARAMS, ids=lambda d: ",".join(f"{k}={v}" for k, v in d.items()) or "defaults")
@pytest.mark.parametrize("algo_name", ALGOS)
def test_stepped_all_resident(mg, pool, algo_name, kw):
    """Every request resident at once (each step sweeps all of them), under sketch
    sizes, modes and limits that change the labels."""
    algo = _algo(mg, algo_name)
    if algo == mg.ALGO_LPA:
        kw = {k: v for k, v in kw.items() if k not in ("aggregation", "max_passes", "k_aggregate")}
    order = [0, 1, 2, 3, 4, 5, 6, 7, 4, 2, 6]
    with mg.Server(algo, 1 << 30, slots=64, stepped=True, **kw) as srv:
        _check_same(mg, algo, pool, srv, order, kw, stepped=True)


@pytest.mark.parametrize("sweeps", [1, 2, 5])
@pytest.mark.parametrize("algo_name", ALGOS)
def test_stepped_sweeps_per_step(mg, pool, algo_name, sweeps):
    """Steps of one, two or five sweeps: levels end inside or across steps, graphs
    freeze within a step and resume in the next, joining and ending at any point."""
    algo = _algo(mg, algo_name)
    order = [4, 0, 5, 3, 1, 7, 2, 6, 4, 4, 0]
    with mg.Server(algo, 1 << 30, slots=5, stepped=True, sweeps_per_step=sweeps) as srv:
        _check_same(mg, algo, pool, srv, order, {}, stepped=True)


def test_stepped_lpa_one_scan(mg, pool):
    kw = dict(one_scan=1, k=2)
    with mg.Server(mg.ALGO_LPA, 1 << 30, slots=8, stepped=True, **kw) as srv:
        _check_same(mg, mg.ALGO_LPA, pool, srv, [3, 4, 0, 1, 2, 5, 6, 7], kw, stepped=True)


def test_memory_bound_admission(mg, pool):
    """An arena that holds one large request at a time still serves everything, in
    arrival order, and never exceeds its size."""
    import ctypes as ct
    p = mg.params(mg.ALGO_LOUVAIN)
    need = max(int(mg.lib().mgcd_workspace_bytes(mg.ALGO_LOUVAIN, g.n, g.nnz, ct.byref(p)))
               for g in pool)
    arena = (need + 255) // 256 * 256 + 4096
    with mg.Server(mg.ALGO_LOUVAIN, arena, slots=4) as srv:
        _check_same(mg, mg.ALGO_LOUVAIN, pool, srv, [4, 4, 3, 4, 0, 1], {})
        assert srv.info()["peak_bytes"] <= arena


@pytest.mark.parametrize("stepped", [False, True], ids=["calls", "steps"])
def test_staggered_arrivals(mg, pool, stepped):
    """Requests submitted while others run are admitted as slots free up."""
    solo = _solo(mg, mg.ALGO_LOUVAIN, pool[4], {})
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 30, slots=2, stepped=stepped) as srv:
        first = [srv.submit(pool[4]) for _ in range(3)]
        states = {srv.poll(t) for t in first}
        assert states <= {"waiting", "running", "done"}
        time.sleep(0.01)
        later = [srv.submit(pool[4]) for _ in range(3)]
        for t in first + later:
            lab, st, tm = srv.wait(t)
            np.testing.assert_array_equal(lab.cpu().numpy(), solo[0])
        with pytest.raises(mg.MgcdError):
            srv.poll(first[0])  # released by wait


@pytest.mark.parametrize("stepped", [False, True], ids=["calls", "steps"])
def test_oversized_request_rejected(mg, pool, stepped):
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 16, slots=1, stepped=stepped) as srv:
        with pytest.raises(mg.MgcdError) as e:
            srv.submit(pool[4])
        assert e.value.code == -4


def test_served_matches_oracle(mg, pool):
    """One served result against the oracle directly (labels are canonical on both)."""
    g = _pool()[2]
    want, _ = oracle.louvain(g, mode=oracle.MODE_ALG1, k=8, chunk_len=128)
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 28, slots=2) as srv:
        t = srv.submit(pool[2])
        lab, _, _ = srv.wait(t)
    np.testing.assert_array_equal(lab.cpu().numpy(), want)


@pytest.mark.parametrize("algo_name", ALGOS)
def test_stepped_matches_oracle(mg, pool, algo_name):
    """Every request of a step-served mix against the oracle directly."""
    algo = _algo(mg, algo_name)
    run = {"lpa": oracle.lpa, "louvain": oracle.louvain, "leiden": oracle.leiden}[algo_name]
    k = 16 if algo_name == "leiden" else 8
    graphs = _pool()
    with mg.Server(algo, 1 << 30, slots=16, stepped=True) as srv:
        tickets = [(srv.submit(pool[i]), i) for i in range(len(pool))]
        for t, i in tickets:
            lab, st, _ = srv.wait(t)
            want, ost = run(graphs[i], mode=oracle.MODE_ALG1, k=k, chunk_len=128)
            np.testing.assert_array_equal(lab.cpu().numpy(), want)
            assert st["iterations"] == ost.iterations and st["passes"] == ost.passes


def test_stepped_memory_bound_admission(mg, pool):
    """A blocks part that holds one large request at a time still serves everything
    in arrival order; bytes in use never exceed it."""
    import ctypes as ct
    p = mg.params(mg.ALGO_LOUVAIN)
    L = mg.lib()
    big = max(pool, key=lambda g: g.nnz)
    shared = 64 << 20
    # one block of the largest request and a little more (blocks are 256-byte aligned)
    need = int(L.mgcd_workspace_bytes(mg.ALGO_LOUVAIN, big.n, big.nnz, ct.byref(p)))
    with mg.Server(mg.ALGO_LOUVAIN, shared + need, slots=8, stepped=True, shared_bytes=shared) as srv:
        _check_same(mg, mg.ALGO_LOUVAIN, pool, srv, [4, 4, 3, 4, 0, 1, 7], {}, stepped=True)
        assert srv.info()["peak_bytes"] <= need


def test_stepped_one_resident(mg, pool):
    with mg.Server(mg.ALGO_LEIDEN, 1 << 30, slots=1, stepped=True) as srv:
        _check_same(mg, mg.ALGO_LEIDEN, pool, srv, [2, 5, 4, 7], {}, stepped=True)
        assert srv.info()["peak_bytes"] > 0


def test_stepped_bad_graph_fails_alone(mg, pool):
    """With validation on, a malformed request fails with its own error while the
    requests resident beside it finish with their own results."""
    import torch
    g = _pool()[1]
    bad = mg.to_device(g)
    idx = bad.indices.clone()
    idx[3] = g.n + 5  # out of range
    bad = mg.DeviceGraph(bad.offsets, idx, bad.weights)
    kw = dict(validate=1)
    solo = [_solo(mg, mg.ALGO_LOUVAIN, pool[i], kw) for i in (3, 4)]
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 30, slots=8, stepped=True, **kw) as srv:
        t3 = srv.submit(pool[3])
        tb = srv.submit(bad)
        t4 = srv.submit(pool[4])
        with pytest.raises(mg.MgcdError) as e:
            srv.wait(tb)
        assert e.value.code == -2
        for t, want in ((t3, solo[0]), (t4, solo[1])):
            lab, st, _ = srv.wait(t)
            np.testing.assert_array_equal(lab.cpu().numpy(), want[0])
    torch.cuda.synchronize()


def test_stepped_serving_stream(mg):
    """Distinct R-MAT requests (the serving workload's generator, small scales), all
    submitted at once: each equals its own call."""
    reqs = synth.serving_stream(count=12, smin=8, smax=12, deg=16, seed=11)
    graphs = [mg.to_device(synth.rmat(s, 8, seed=gs)) for _, s, gs in reqs]
    solo = [_solo(mg, mg.ALGO_LOUVAIN, g, {}) for g in graphs]
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 30, slots=6, stepped=True) as srv:
        tickets = [srv.submit(g) for g in graphs]
        for t, want in zip(tickets, solo):
            lab, st, _ = srv.wait(t)
            np.testing.assert_array_equal(lab.cpu().numpy(), want[0])
            assert st["iterations"] == want[1]["iterations"]


def test_stepped_step_stats(mg, pool):
    """The engine's counters: steps, sweeps and transitions happened; frozen rows are
    never more than the swept ones; a whole-call server reports zeros."""
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 30, slots=8, stepped=True, sweeps_per_step=3) as srv:
        ts = [srv.submit(pool[i]) for i in (0, 1, 2, 3, 4, 5)]
        passes = 0
        for t in ts:
            _, st, _ = srv.wait(t)
            passes += st["passes"]
        c = srv.step_stats()
    assert c["steps"] >= 1 and c["packs"] >= 1
    assert c["sweeps"] == 3 * c["steps"] and c["sweeps_moving"] <= c["sweeps"]
    assert 0 < c["rows_moving"] <= c["rows_swept"]
    assert c["transitions"] == passes  # every level of every request ends once
    assert min(c["s_pack"], c["s_sweep"], c["s_phase"], c["s_admit"]) >= 0.0 and c["s_admit"] > 0.0
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 28, slots=2) as srv:
        assert all(v == 0 for v in srv.step_stats().values())


@pytest.mark.parametrize("stepped", [False, True], ids=["calls", "steps"])
def test_destroy_drains(mg, pool, stepped):
    """Destroying a server with requests still queued or running runs them to
    completion first (their outputs are written) and returns."""
    import torch
    want = _solo(mg, mg.ALGO_LOUVAIN, pool[4], {})[0]
    srv = mg.Server(mg.ALGO_LOUVAIN, 1 << 30, slots=2, stepped=stepped)
    ts = [srv.submit(pool[4]) for _ in range(5)]
    outs = [srv._held[t][1] for t in ts]
    srv.close()
    torch.cuda.synchronize()
    for o in outs:
        np.testing.assert_array_equal(o[:pool[4].n].cpu().numpy(), want)


def test_stepped_rejects_bad_params(mg):
    with pytest.raises(mg.MgcdError) as e:
        mg.Server(mg.ALGO_LOUVAIN, 1 << 24, slots=4, stepped=True, k=3)
    assert e.value.code == -6
    with pytest.raises(mg.MgcdError) as e:
        mg.Server(mg.ALGO_LOUVAIN, 1 << 24, slots=4, stepped=True, one_scan=1)
    assert e.value.code == -6
    with pytest.raises(mg.MgcdError) as e:
        mg.Server(mg.ALGO_LPA, 1 << 24, slots=0, stepped=True)
    assert e.value.code == -1
