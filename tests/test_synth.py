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
