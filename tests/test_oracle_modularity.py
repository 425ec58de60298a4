"""Pins for the oracle's modularity (Section 3.2, Eq. 1) and for the integer form of
delta-modularity (Section 3.2, Eq. 2) that decides every Louvain/Leiden move.
References: closed forms, the networkx library (a black box), brute force."""
import math

import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth
from _graphs import disjoint_cliques, nx_modularity


@pytest.mark.parametrize("r,s", [(2, 3), (3, 4), (5, 5), (8, 3)])
def test_disjoint_cliques_closed_form(r, s):
    g = disjoint_cliques(r, s)
    C = np.repeat(np.arange(r), s).astype(np.int32)
    assert abs(oracle.modularity(g, C) - (1 - 1 / r)) < 1e-12


def test_one_community_and_singletons():
    g = synth.random_small(12, 0.4, 5, seed=3)
    assert abs(oracle.modularity(g, np.zeros(g.n, dtype=np.int32))) < 1e-12
    K = oracle.weighted_degree(g).astype(float)
    W = K.sum()
    exp = -np.sum((K / W) ** 2)
    assert abs(oracle.modularity(g, np.arange(g.n, dtype=np.int32)) - exp) < 1e-12


def test_path3_values():
    g = synth.from_edges(3, [(0, 1), (1, 2)])
    assert abs(oracle.modularity(g, np.array([0, 1, 2], np.int32)) + 0.375) < 1e-12
    assert abs(oracle.modularity(g, np.array([0, 0, 1], np.int32)) + 0.125) < 1e-12


def test_planted_ground_truth_is_070():
    # 12 intra and 4 inter edges per vertex, 20 equal communities:
    # Q = 12/16 - 20 * (1/20)^2 = 0.70.
    g, truth = synth.planted_exact()
    assert abs(oracle.modularity(g, truth) - 0.70) < 1e-12


@pytest.mark.parametrize("seed", range(12))
def test_matches_networkx(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    g = synth.random_small(n, float(rng.uniform(0.1, 0.5)), 8, seed=seed)
    C = rng.integers(0, max(1, n // 3), size=n).astype(np.int32)
    assert abs(oracle.modularity(g, C) - nx_modularity(g, C)) < 1e-12


@pytest.mark.parametrize("seed", range(8))
def test_self_loop_convention_by_aggregation(seed):
    # Exact aggregation of a loop-free graph yields self-loops; the modularity of the
    # aggregate under singletons must equal the networkx value of the original.
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(6, 30))
    g = synth.random_small(n, 0.3, 6, seed=100 + seed)
    C = rng.integers(0, max(1, n // 4), size=n)
    u, D = np.unique(C, return_inverse=True)
    a = oracle.aggregate(g, D.astype(np.int32), len(u), mode=oracle.MODE_EXACT)
    q_agg = oracle.modularity(a, np.arange(len(u), dtype=np.int32))
    assert abs(q_agg - nx_modularity(g, D)) < 1e-12


def _best_move_brute(g, C, i, qfun):
    """Every move of vertex i into a neighbouring community, valued by the
    difference of modularity before and after (Eq. 1 evaluated twice)."""
    q0 = qfun(g, C)
    W = float(oracle.weighted_degree(g).sum())
    best, bestg = int(C[i]), 0.0
    cands = sorted({int(C[j]) for j in g.indices[g.offsets[i]:g.offsets[i + 1]] if j != i})
    for c in cands:
        if c == C[i]:
            continue
        C2 = C.copy()
        C2[i] = c
        gval = (qfun(g, C2) - q0) * W * W / 2.0
        if gval > bestg + 1e-6 or (abs(gval - bestg) <= 1e-6 and gval > 1e-6 and c < best):
            best, bestg = c, gval
    return best, bestg


@pytest.mark.parametrize("seed", range(10))
def test_exact_sweep_matches_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(5, 16))
    g = synth.random_small(n, 0.45, 5, seed=200 + seed)
    C = rng.integers(0, max(1, n // 2), size=n).astype(np.int32)
    Cn, gain = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=oracle.MODE_EXACT)
    for i in range(n):
        best, bg = _best_move_brute(g, C, i, nx_modularity)
        assert abs(gain[i] - bg) < 1e-6
        assert Cn[i] == best


@pytest.mark.parametrize("seed", range(6))
def test_exact_sweep_with_self_loops(seed):
    # Self-loops are left out of K_{i->c} (Appendix A.1); Eq. 2 stays exact because
    # the self-loop terms cancel.  Reference: the (pinned) Eq. 1 value of the
    # oracle, evaluated before and after each move.
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(5, 14))
    g = synth.random_small(n, 0.45, 5, seed=300 + seed, loops=True)
    C = rng.integers(0, max(1, n // 2), size=n).astype(np.int32)
    Cn, gain = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=oracle.MODE_EXACT)
    for i in range(n):
        best, bg = _best_move_brute(g, C, i, oracle.modularity)
        assert abs(gain[i] - bg) < 1e-6
        assert Cn[i] == best


def test_gain_is_an_integer_multiple():
    # dQ = 2G/W^2: one move on the path (hand derivation in golden/path3_louvain.txt).
    g = synth.from_edges(3, [(0, 1), (1, 2)])
    C = np.array([0, 1, 2], np.int32)
    _, gain = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=oracle.MODE_EXACT)
    assert list(gain) == [2, 2, 2]
    assert math.isclose(2 * gain[0] / 16, -0.125 - -0.375)
