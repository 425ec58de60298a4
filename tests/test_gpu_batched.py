"""Batched runs on the GPU: per-graph validation and weight limits, and a batch whose
entries exceed 2^31 (every graph equal to its own plain call, sampled graphs equal
to the oracle).  Run on an MI355X only."""
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


def _bad_copies():
    """(name, graphs) where graph 1 of 3 breaks one rule; each break would still look
    valid in the packed union (an index into a neighbouring graph, a negative index
    into the previous one, offsets that do not start at 0 or end at nnz)."""
    base = [synth.random_small(30, 0.2, 4, seed=s) for s in (1, 2, 3)]
    out = []

    def variant(name, fix):
        gs = [synth.CSR(g.offsets.copy(), g.indices.copy(), g.weights.copy()) for g in base]
        fix(gs[1])
        out.append((name, gs))
    variant("index n_g (a vertex of graph 2 in the union)", lambda g: g.indices.__setitem__(0, g.n))
    variant("index -1 (the last vertex of graph 0 in the union)", lambda g: g.indices.__setitem__(3, -1))
    variant("offsets[0] != 0", lambda g: g.offsets.__setitem__(0, 1))
    variant("offsets[n] != nnz", lambda g: g.offsets.__setitem__(g.n, g.nnz - 1))
    variant("weight 0", lambda g: g.weights.__setitem__(5, 0))
    return base, out


def test_batched_validation_per_graph(mg):
    base, cases = _bad_copies()
    for algo in (mg.ALGO_LPA, mg.ALGO_LOUVAIN):
        labs, _, _ = mg.run_batched(algo, [mg.to_device(g) for g in base], validate=1)
        for name, gs in cases:
            with pytest.raises(mg.MgcdError) as ei:
                mg.run_batched(algo, [mg.to_device(g) for g in gs], validate=1)
            assert ei.value.code == -2 and "graph 1" in str(ei.value), name


def test_batched_row_weight_wrap_is_an_overflow(mg):
    # graph 1: vertex 0 carries two self-loop entries of 2^31 and 2^31 + 1; its row sum
    # (2^32 + 1) wraps to 1 in 32 bits, so only the exact total shows the overflow
    ok = synth.random_small(20, 0.2, 4, seed=7)
    off = np.array([0, 2, 2], np.int64)
    heavy = synth.CSR(off, np.array([0, 0], np.int32), np.array([1 << 31, (1 << 31) + 1], np.uint32))
    with pytest.raises(mg.MgcdError) as ei:
        mg.run_batched(mg.ALGO_LOUVAIN, [mg.to_device(ok), mg.to_device(heavy)])
    assert ei.value.code == -3


@pytest.mark.timeout(600)
def test_batched_beyond_2_31_entries(mg):
    """68 copies of the R-MAT 2^20 graph (the same device arrays each time), then an
    R-MAT 2^19 graph across entry 2^31 of the union, then three planted graphs wholly
    beyond it: every graph's labels equal its plain call's, and the distinct graphs
    equal the oracle's."""
    import torch
    big = synth.rmat(scale=20, edge_factor=16, seed=2, device="cuda")
    mid = synth.rmat(scale=19, edge_factor=16, seed=11, device="cuda")
    tail = [synth.planted_exact(n_comm=6, comm_size=40 + 10 * s, seed=30 + s)[0] for s in range(3)]
    dbig = mg.to_device(big)
    graphs = [dbig] * 68 + [mg.to_device(mid)] + [mg.to_device(g) for g in tail]
    bases = np.cumsum([0] + [g.nnz for g in graphs])
    assert bases[68] < (1 << 31) < bases[69] and bases[-1] > (1 << 31)
    print(f"batch of {len(graphs)} graphs, {bases[-1]} entries", flush=True)
    for algo, fn, ofn in ((mg.ALGO_LPA, mg.lpa, oracle.lpa),
                          (mg.ALGO_LOUVAIN, mg.louvain, oracle.louvain)):
        labs, per, _ = mg.run_batched(algo, graphs, k=8)
        solo_big, st_big = fn(dbig, k=8)
        for x in range(68):
            assert torch.equal(labs[x], solo_big), f"copy {x}"
            assert per[x]["iterations"] == st_big["iterations"]
        for x, g in zip(range(68, len(graphs)), [mid] + tail):
            solo, st = fn(graphs[x], k=8)
            assert torch.equal(labs[x], solo), f"graph {x}"
            elab, est = ofn(g, k=8)
            assert np.array_equal(labs[x].cpu().numpy(), elab), f"graph {x} vs oracle"
            assert per[x]["iterations"] == est.iterations
        elab, _ = ofn(big, k=8)
        assert np.array_equal(solo_big.cpu().numpy(), elab)
        print(f"algo {algo}: batch equal to plain calls and the oracle", flush=True)
        del labs
        torch.cuda.empty_cache()
