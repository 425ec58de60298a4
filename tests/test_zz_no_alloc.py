"""modularity_noalloc: modularity() without a caller workspace, working in the
library's fixed per-device scratch.  Checked against modularity() (bit-identical: the
same kernels and reductions) and the oracle (Eq. 1, relative 1e-9), on consecutive
calls whose second input is smaller than the first, plus the size limit."""
import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth


def _close(q, ref):
    return abs(q - ref) <= 1e-9 * max(abs(ref), 1e-12) + 1e-15


@pytest.mark.gpu
def test_noalloc_equals_modularity_on_consecutive_calls():
    import torch
    import paper_2411_02268_amd as mg
    big = synth.rmat(scale=17, edge_factor=16, seed=21)
    small, _ = synth.planted_exact(n_comm=6, comm_size=40, seed=3)
    gen = torch.Generator(device="cpu").manual_seed(5)
    for g in (big, small):  # the second call's graph is smaller than the first's
        dg = mg.to_device(g)
        lab, _ = mg.louvain(dg, k=8)
        rnd = torch.randint(0, g.n, (g.n,), generator=gen, dtype=torch.int32).to(lab.device)
        for labels in (lab, rnd):
            q_ref = mg.modularity(dg, labels)
            q = mg.modularity_noalloc(dg, labels)
            assert q == q_ref
            assert _close(q, oracle.modularity(g, labels.cpu().numpy()))
        print(f"noalloc n={g.n} nnz={g.nnz}: equal to modularity()", flush=True)


@pytest.mark.gpu
def test_noalloc_limits_and_edges():
    import torch
    import paper_2411_02268_amd as mg
    dev = "cuda"
    # the largest accepted vertex count (no edges: Q = 0), then one more vertex
    nmax = mg.NOALLOC_MAX_VERTICES
    for n, ok in ((nmax, True), (nmax + 1, False)):
        g = mg.DeviceGraph(torch.zeros(n + 1, dtype=torch.int64, device=dev),
                           torch.zeros(4, dtype=torch.int32, device=dev)[:0],
                           torch.zeros(4, dtype=torch.int32, device=dev)[:0])
        lab = torch.arange(n, dtype=torch.int32, device=dev)
        if ok:
            assert mg.modularity_noalloc(g, lab) == 0.0
        else:
            with pytest.raises(mg.MgcdError) as e:
                mg.modularity_noalloc(g, lab)
            assert e.value.code == -4 and "at most" in str(e.value)
    # labels out of range are refused; an empty graph has Q = 0
    g, _ = synth.planted_exact(n_comm=4, comm_size=30, seed=2)
    dg = mg.to_device(g)
    bad = torch.full((g.n,), g.n, dtype=torch.int32, device=dev)
    with pytest.raises(mg.MgcdError) as e:
        mg.modularity_noalloc(dg, bad)
    assert e.value.code == -1
    lab, _ = mg.lpa(dg)
    assert mg.modularity_noalloc(dg, lab) == mg.modularity(dg, lab)
    empty = mg.DeviceGraph(torch.zeros(1, dtype=torch.int64, device=dev),
                           torch.zeros(4, dtype=torch.int32, device=dev)[:0],
                           torch.zeros(4, dtype=torch.int32, device=dev)[:0])
    assert mg.modularity_noalloc(empty, torch.zeros(0, dtype=torch.int32, device=dev)) == 0.0
