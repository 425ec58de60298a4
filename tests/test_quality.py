"""NMI against the library implementation in scikit-learn and closed forms."""
import numpy as np
import pytest

from paper_2411_02268_amd.quality import nmi


def test_closed_forms():
    x = np.repeat(np.arange(5), 7)
    assert nmi(x, x) == pytest.approx(1.0)
    perm = np.random.default_rng(0).permutation(5)
    assert nmi(x, perm[x] + 100) == pytest.approx(1.0)          # renaming
    assert nmi(np.zeros(35), np.arange(35)) == pytest.approx(0.0)  # one vs singletons
    assert nmi(np.zeros(9), np.zeros(9)) == 1.0
    # two halves vs four quarters: I = log 2, H(A) = log 2, H(B) = log 4 -> 2/3
    a = np.repeat([0, 1], 4)
    b = np.repeat([0, 1, 2, 3], 2)
    assert nmi(a, b) == pytest.approx(2 * np.log(2) / (np.log(2) + np.log(4)))


@pytest.mark.parametrize("seed", range(5))
def test_matches_scikit_learn(seed):
    from sklearn.metrics import normalized_mutual_info_score
    rng = np.random.default_rng(seed)
    n = int(rng.integers(10, 400))
    a = rng.integers(0, int(rng.integers(1, 30)), size=n)
    b = np.where(rng.random(n) < 0.6, a, rng.integers(0, 20, size=n))
    assert nmi(a, b) == pytest.approx(normalized_mutual_info_score(a, b), abs=1e-12)
