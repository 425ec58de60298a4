"""The seeded input generators: the torch-sorted CSR build (used for the largest
graphs, on the GPU) gives the same CSR as the numpy build."""
import numpy as np
import pytest

from paper_2411_02268_amd import synth


@pytest.mark.parametrize("make", [
    lambda d: synth.rmat(scale=12, edge_factor=8, seed=5, device=d),
    lambda d: synth.chung_lu(n=1 << 13, avg_deg=20, seed=6, device=d),
])
def test_torch_sorted_build_equals_numpy(make):
    a, b = make(None), make("cpu")
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.indices, b.indices) and b.indices.dtype == np.int32
    assert np.array_equal(a.weights, b.weights) and b.weights.dtype == np.uint32
    # symmetric, no self-loops, rows sorted
    for i in range(0, a.n, 97):
        row = a.indices[a.offsets[i]:a.offsets[i + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == i)


def test_rmat_torch_is_a_valid_undirected_csr():
    """The torch-drawn R-MAT of the serving stream: symmetric entries with equal
    weights, rows sorted without duplicates or self-loops, weights in [1, 8], and the
    same graph for the same seed (different for another)."""
    import torch
    off, idx, w = synth.rmat_torch(11, 8, seed=7, device="cpu")
    o, ii, ww = off.numpy(), idx.numpy(), w.numpy().view(np.uint32)
    n = o.shape[0] - 1
    assert n == 2048 and o[0] == 0 and o[-1] == ii.shape[0]
    rows = np.repeat(np.arange(n), np.diff(o))
    assert not np.any(rows == ii)
    for i in range(n):
        assert np.all(np.diff(ii[o[i]:o[i + 1]]) > 0)
    assert ww.min() >= 1 and ww.max() <= 8
    fwd = set(zip(rows.tolist(), ii.tolist(), ww.tolist()))
    assert fwd == set(zip(ii.tolist(), rows.tolist(), ww.tolist()))
    off2, idx2, w2 = synth.rmat_torch(11, 8, seed=7, device="cpu")
    assert torch.equal(off, off2) and torch.equal(idx, idx2) and torch.equal(w, w2)
    _, idx3, _ = synth.rmat_torch(11, 8, seed=8, device="cpu")
    assert idx3.shape != idx.shape or not torch.equal(idx3, idx)


@pytest.mark.parametrize("make", [
    lambda: synth.road_like(96, seed=4),
    lambda: synth.kmer_like(20000, seed=5),
])
def test_low_degree_classes(make):
    """Road- and k-mer-like stand-ins: symmetric unit-weight CSRs, rows sorted without
    self-loops or duplicates, about 2.1 entries per vertex (the |E|/|V| of the paper's
    road and k-mer graphs), mostly degree-2 vertices."""
    g = make()
    o, ii, ww = g.offsets, g.indices, g.weights
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(o))
    assert not np.any(rows == ii)
    assert np.all(ww == 1)
    key = rows.astype(np.int64) * n + ii
    assert np.all(np.diff(key) > 0)  # sorted rows, no duplicates
    rev = ii.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(rev), key)  # symmetric
    assert 2.0 <= g.nnz / n <= 2.25
    deg = np.diff(o)
    assert np.mean(deg == 2) > 0.6


def test_road_like_device_sort_equals_host():
    a, b = synth.road_like(80, seed=9), synth.road_like(80, seed=9, device="cpu")
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.indices, b.indices)
    assert np.array_equal(a.weights, b.weights)
