"""Ground-truth scoring of a partition against a planted one (host side).

Normalised mutual information (Danon et al. 2005), as the arithmetic-mean
normalisation 2 I(A;B) / (H(A) + H(B)): 1 for equal partitions (up to renaming), 0
for independent ones.  Not part of the device path: it scores results that the
library has already produced.
"""
from __future__ import annotations

import numpy as np


def nmi(a, b) -> float:
    """NMI of two labelings of the same vertices (any integer labels)."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    if a.shape != b.shape:
        raise ValueError("labelings differ in length")
    n = a.shape[0]
    if n == 0:
        return 1.0
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    na, nb = int(ai.max()) + 1, int(bi.max()) + 1
    pa = np.bincount(ai, minlength=na) / n
    pb = np.bincount(bi, minlength=nb) / n
    pairs, cnt = np.unique(ai.astype(np.int64) * nb + bi, return_counts=True)
    pab = cnt / n
    x, y = pairs // nb, pairs % nb
    mi = float(np.sum(pab * np.log(pab / (pa[x] * pb[y]))))
    ha = float(-np.sum(pa * np.log(pa)))
    hb = float(-np.sum(pb * np.log(pb)))
    if ha + hb == 0.0:
        return 1.0  # both partitions are one community
    return max(0.0, 2.0 * mi / (ha + hb))
