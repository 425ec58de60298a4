"""Serving (continuous batching): every request's result equals the same call made
alone, whatever else is resident; admission respects the arena; errors surface."""
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


def _check_same(mg, algo, pool, server, order, kw):
    solo = [_solo(mg, algo, dg, kw) for dg in pool]
    tickets = [(server.submit(pool[i]), i) for i in order]
    for t, i in tickets:
        lab, st, tm = server.wait(t)
        np.testing.assert_array_equal(lab.cpu().numpy(), solo[i][0])
        for key in ("iterations", "passes", "communities", "edges_scanned"):
            assert st[key] == solo[i][1][key], key
        assert tm[0] <= tm[1] <= tm[2]


@pytest.mark.parametrize("algo_name", ["louvain", "lpa", "leiden"])
def test_alone_equals_mixed(mg, pool, algo_name):
    algo = {"lpa": mg.ALGO_LPA, "louvain": mg.ALGO_LOUVAIN, "leiden": mg.ALGO_LEIDEN}[algo_name]
    kw = {}
    order = [4, 0, 5, 3, 1, 7, 2, 6, 4, 4, 0]
    with mg.Server(algo, 1 << 30, slots=4, **kw) as srv:
        _check_same(mg, algo, pool, srv, order, kw)
        info = srv.info()
        assert info["waiting"] == 0 and info["running"] == 0 and info["bytes_in_use"] == 0


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


def test_staggered_arrivals(mg, pool):
    """Requests submitted while others run are admitted as slots free up."""
    solo = _solo(mg, mg.ALGO_LOUVAIN, pool[4], {})
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 30, slots=2) as srv:
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


def test_oversized_request_rejected(mg, pool):
    with mg.Server(mg.ALGO_LOUVAIN, 1 << 16, slots=1) as srv:
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
