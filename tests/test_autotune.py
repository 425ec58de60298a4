"""Autotuner: the selection rules (CPU), and on the GPU that the tuned k reproduces
the oracle bit for bit and that schedule knobs never change labels."""
import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import autotune, synth


def test_choose_k_fastest_that_meets_quality():
    table = {1: (0.90, 1.0), 2: (0.995, 2.0), 4: (0.999, 1.5), 8: (1.0, 3.0)}
    assert autotune.choose_k(table, 0.99) == (4, True)
    assert autotune.choose_k(table, 0.9995) == (8, True)


def test_choose_k_best_quality_when_none_meets():
    table = {1: (0.50, 1.0), 2: (0.70, 2.0), 4: (0.70, 1.5)}
    assert autotune.choose_k(table, 0.99) == (4, False)


def test_choose_fastest():
    assert autotune.choose_fastest({8: 2.0, 16: 1.0, 32: 1.0}) == 16


def test_params_file_roundtrip(tmp_path):
    tuned = {"algo": 1, "mode": 1, "k": 4, "k_aggregate": 4, "chunk_len": 128, "row_lanes": 16,
             "short_rows": 2, "exact_small": 32, "exact_lds": 512, "exact_lds_big": 4096, "report": {}}
    path = str(tmp_path / "p.json")
    autotune.save(tuned, path)
    back = autotune.load(path)
    assert autotune.run_kwargs(back) == {k: tuned[k] for k in autotune.PARAM_KEYS}
    ex = autotune.run_kwargs(back, exact=True)
    assert ex["mode"] == 0 and "short_rows" not in ex


@pytest.fixture(scope="module")
def mg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_02268_amd as m
    m.lib()
    return m


@pytest.mark.gpu
@pytest.mark.parametrize("algo_name,batched", [("louvain", False), ("lpa", False),
                                               ("louvain", True)])
def test_tuned_params_match_oracle(mg, algo_name, batched):
    host = [synth.planted_exact(n_comm=8, comm_size=60, seed=11)[0],
            synth.rmat(scale=11, edge_factor=8, seed=12),
            synth.chung_lu(n=1 << 11, avg_deg=20, seed=13)]
    sample = [mg.to_device(g) for g in host]
    algo = mg.ALGO_LOUVAIN if algo_name == "louvain" else mg.ALGO_LPA
    tuned = autotune.tune(mg, sample, algo, repeats=1, batched=batched, chunk_len=16)
    assert tuned["k"] in autotune.SKETCH_K
    kw = autotune.run_kwargs(tuned)
    ofn = oracle.louvain if algo == mg.ALGO_LOUVAIN else oracle.lpa
    fn = mg.louvain if algo == mg.ALGO_LOUVAIN else mg.lpa
    for g, dg in zip(host, sample):
        want, _ = ofn(g, mode=oracle.MODE_ALG1, k=tuned["k"], chunk_len=16)
        got, _ = fn(dg, **kw)
        np.testing.assert_array_equal(got.cpu().numpy(), want)
        want_x, _ = ofn(g, mode=oracle.MODE_EXACT, k=tuned["k"], chunk_len=16)
        got_x, _ = fn(dg, **autotune.run_kwargs(tuned, exact=True))
        np.testing.assert_array_equal(got_x.cpu().numpy(), want_x)


@pytest.mark.gpu
@pytest.mark.parametrize("rl", [1, 2, 4, 8, 16, 32, 64])
def test_row_lanes_never_change_results(mg, rl):
    g = synth.rmat(scale=11, edge_factor=8, seed=3)
    dg = mg.to_device(g)
    for L in (2, 16):
        want, _ = oracle.louvain(g, mode=oracle.MODE_ALG1, k=8, chunk_len=L)
        got, _ = mg.louvain(dg, k=8, chunk_len=L, row_lanes=rl)
        np.testing.assert_array_equal(got.cpu().numpy(), want)


@pytest.mark.gpu
@pytest.mark.parametrize("tiers", [(0, 0, 0), (1, 2, 3), (64, 64, 64), (8, 512, 4096),
                                   (32, 100, 200)])
def test_exact_tiers_never_change_results(mg, tiers):
    g = synth.rmat(scale=11, edge_factor=8, seed=4)
    dg = mg.to_device(g)
    want, _ = oracle.louvain(g, mode=oracle.MODE_EXACT, k=8, chunk_len=128)
    got, _ = mg.louvain(dg, mode=mg.MODE_EXACT, exact_small=tiers[0], exact_lds=tiers[1],
                        exact_lds_big=tiers[2])
    np.testing.assert_array_equal(got.cpu().numpy(), want)


@pytest.mark.gpu
def test_bad_schedule_knobs_rejected(mg):
    dg = mg.to_device(synth.rmat(scale=8, edge_factor=4, seed=1))
    for kw in ({"row_lanes": 3}, {"row_lanes": 128}, {"exact_lds": 513},
               {"exact_lds_big": 5000}, {"exact_small": -1}):
        with pytest.raises(mg.MgcdError):
            mg.louvain(dg, **kw)
