"""Full-size parity on the web-like workload: Leiden, MG k=16, on the Chung-Lu graph
of 2^24 vertices (average degree 32, exponent 2.1, weights in [1, 4]; about 5.35e8
CSR entries).  Labels, sweeps and passes bit-exact with the oracle; modularity within
a relative 1e-9.  Run on an MI355X only (the oracle takes a minute or two on the
host)."""
import time

import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1000)
def test_chung_lu_2_24_leiden_k16():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_02268_amd as mg
    t0 = time.time()
    g = synth.chung_lu(n=1 << 24, avg_deg=32, seed=3, device="cuda")
    print(f"Chung-Lu 2^24: nnz={g.nnz} generated in {time.time() - t0:.1f}s", flush=True)
    assert g.nnz > 5e8
    dg = mg.to_device(g)
    lab, st = mg.leiden(dg, k=16)
    q = mg.modularity(dg, lab)
    got = lab.cpu().numpy()
    del dg, lab
    torch.cuda.empty_cache()
    print(f"GPU: {st['iterations']} sweeps, {st['passes']} passes, Q={q:.6f}", flush=True)
    t0 = time.time()
    elab, est = oracle.leiden(g, k=16)
    print(f"oracle in {time.time() - t0:.1f}s: {est.iterations} sweeps, {est.passes} passes", flush=True)
    assert np.array_equal(got, elab)
    assert st["iterations"] == est.iterations and st["passes"] == est.passes
    assert st["communities"] == est.communities
    eq = oracle.modularity(g, elab)
    assert abs(q - eq) <= 1e-9 * abs(eq)
