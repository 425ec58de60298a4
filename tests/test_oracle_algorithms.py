"""Pins for the oracle's LPA, Louvain and Leiden drivers (Sections 3.3-3.5, 4.1-4.3).
References: hand traces, closed forms, brute-force optimum on tiny graphs,
textbook LPA, invariants of refinement and aggregation, and the equality of the
MG and exact modes when k covers every key (no subtraction can happen)."""
import os
from collections import defaultdict

import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth
from _graphs import (disjoint_cliques, nx_modularity, partition_labels, set_partitions,
                     clique_edges)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "path3_louvain.txt")
BIGK = dict(k=1024, k_aggregate=1024)


# ---------------------------------------------------------------------------------
# LPA
# ---------------------------------------------------------------------------------

def textbook_lpa_step(g, C):
    """One synchronous LPA step (Raghavan et al.): the label of largest total weight
    among the neighbours (self excluded), the lowest on ties; none -> keep."""
    Cn = C.copy()
    for i in range(g.n):
        tot = defaultdict(int)
        for e in range(g.offsets[i], g.offsets[i + 1]):
            j = int(g.indices[e])
            if j != i:
                tot[int(C[j])] += int(g.weights[e])
        if tot:
            m = max(tot.values())
            Cn[i] = min(c for c, v in tot.items() if v == m)
    return Cn


@pytest.mark.parametrize("seed", range(6))
def test_lpa_exact_step_is_textbook(seed):
    rng = np.random.default_rng(seed)
    g = synth.random_small(30, 0.2, 4, seed=seed, loops=True)
    C = rng.integers(0, 8, size=g.n).astype(np.int32)
    Cn, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_EXACT)
    assert np.array_equal(Cn, textbook_lpa_step(g, C))


def test_lpa_closed_forms():
    k4 = synth.from_edges(4, clique_edges(range(4)))
    lab, st = oracle.lpa(k4, mode=oracle.MODE_EXACT)
    assert list(lab) == [0, 0, 0, 0] and st.iterations == 3
    tri = synth.from_edges(3, clique_edges(range(3)))
    lab, st = oracle.lpa(tri, mode=oracle.MODE_EXACT)
    assert list(lab) == [0, 0, 0] and st.iterations == 3
    # K2 swaps labels every sweep (synchronous updates) until the 20-sweep cap
    k2 = synth.from_edges(2, [(0, 1)])
    lab, st = oracle.lpa(k2, mode=oracle.MODE_EXACT)
    assert st.iterations == 20 and list(lab) == [0, 1]
    cl = disjoint_cliques(4, 5)
    for mode in (oracle.MODE_EXACT, oracle.MODE_ALG1):
        lab, _ = oracle.lpa(cl, mode=mode)
        assert list(lab) == list(np.repeat(np.arange(4), 5))


def test_lpa_mg_step_uses_sketch_candidates():
    # MG mode: pass 1 candidates from the (pinned) sketch of the stream of neighbour
    # labels, self excluded; pass 2 exact weights; largest weight, lowest label.
    rng = np.random.default_rng(7)
    g = synth.random_small(60, 0.3, 6, seed=7, loops=True)
    C = rng.integers(0, 20, size=g.n).astype(np.int32)
    k = 3
    Cn, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_ALG1, k=k, chunk_len=5)
    for i in range(g.n):
        row = [(int(C[j]), int(w)) for j, w in zip(g.indices[g.offsets[i]:g.offsets[i + 1]],
                                                   g.weights[g.offsets[i]:g.offsets[i + 1]])]
        # chunk positions count the self entry; it only carries no weight
        keys = [c if j != i else 0 for (c, _), j in zip(row, g.indices[g.offsets[i]:g.offsets[i + 1]])]
        use = [j != i for j in g.indices[g.offsets[i]:g.offsets[i + 1]]]
        # rebuild the stream chunk by chunk, the self entry skipped inside its chunk
        chunks = [list(range(s, min(s + 5, len(row)))) for s in range(0, len(row), 5)]
        sketches = []
        for ch in chunks:
            kk = [keys[e] for e in ch if use[e]]
            ww = [row[e][1] for e in ch if use[e]]
            sketches.append(oracle.sketch_stream(kk, ww, k=k))
        while len(sketches) > 1:
            nxt = [oracle.mg_merge(sketches[x], sketches[x + 1], k)
                   for x in range(0, len(sketches) - 1, 2)]
            if len(sketches) % 2:
                nxt.append(sketches[-1])
            sketches = nxt
        sk = sketches[0] if sketches else {}
        tot = defaultdict(int)
        for (c, w), u in zip(row, use):
            if u:
                tot[c] += w
        if not sk:
            assert Cn[i] == C[i]
            continue
        m = max(tot[c] for c in sk)
        assert Cn[i] == min(c for c in sk if tot[c] == m)


def _star(weights, labels):
    """Vertex 0 joined to vertices 1..len(weights) with the given weights; C[j] =
    labels[j - 1] for the leaves, C[0] = 0."""
    n = 1 + len(weights) + 16
    u = np.zeros(len(weights), dtype=np.int64)
    v = np.arange(1, len(weights) + 1, dtype=np.int64)
    g = synth.csr_from_undirected(n, u, v, w=np.asarray(weights, dtype=np.uint32))
    C = np.arange(n, dtype=np.int32)
    C[0] = 0
    C[1:1 + len(labels)] = labels
    return g, C


def test_lpa_one_scan_hand_trace():
    # Vertex 0's stream in CSR order: (a,5) (b,1) (c,5) (a,1) (b,3), k = 2.
    # Algorithm 1: {a:5} -> {a:5, b:1} -> c misses a full sketch: a and b drop to 0
    # and c is dropped -> a revived with 1 -> b revived with 3: sketch {a:1, b:3}.
    # 1-scan (Section 4.3) takes the largest sketch value: b.  The second pass finds
    # K_{0->a} = 6 > K_{0->b} = 4: a.
    a, b, c = 10, 11, 12
    g, C = _star([5, 1, 5, 1, 3], [a, b, c, a, b])
    assert oracle.sketch_stream([a, b, c, a, b], [5, 1, 5, 1, 3], k=2) == {a: 1, b: 3}
    one, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_ALG1, k=2, one_scan=1)
    two, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_ALG1, k=2, one_scan=0)
    assert one[0] == b and two[0] == a
    # equal sketch values: the lower label
    g, C = _star([2, 2], [b, a])
    one, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_ALG1, k=2, one_scan=1)
    assert one[0] == a


@pytest.mark.parametrize("mode", [oracle.MODE_ALG1, oracle.MODE_UNCOND, oracle.MODE_STD])
def test_lpa_one_scan_takes_largest_sketch_value(mode):
    # every vertex: the label of the largest value of its (pinned) merged sketch,
    # lowest on ties; an empty sketch keeps the label
    rng = np.random.default_rng(11)
    g = synth.random_small(60, 0.3, 6, seed=11, loops=True)
    C = rng.integers(0, 20, size=g.n).astype(np.int32)
    k, L = 3, 5
    Cn, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=mode, k=k, chunk_len=L, one_scan=1)
    for i in range(g.n):
        lo, hi = g.offsets[i], g.offsets[i + 1]
        js, ws = g.indices[lo:hi], g.weights[lo:hi]
        sketches = []
        for s0 in range(0, hi - lo, L):
            kk = [int(C[j]) for j in js[s0:s0 + L] if j != i]
            ww = [int(w) for j, w in zip(js[s0:s0 + L], ws[s0:s0 + L]) if j != i]
            sketches.append(oracle.sketch_stream(kk, ww, mode=mode, k=k))
        while len(sketches) > 1:
            nxt = [oracle.mg_merge(sketches[x], sketches[x + 1], k)
                   for x in range(0, len(sketches) - 1, 2)]
            if len(sketches) % 2:
                nxt.append(sketches[-1])
            sketches = nxt
        sk = sketches[0] if sketches else {}
        if not sk:
            assert Cn[i] == C[i]
            continue
        m = max(sk.values())
        assert Cn[i] == min(c for c, v in sk.items() if v == m)


def test_lpa_one_scan_equals_two_scan_when_sketch_is_exact():
    # k covering every key: the sketch values are the exact weights (no subtraction)
    g = synth.random_small(80, 0.2, 5, seed=3)
    a, sa = oracle.lpa(g, one_scan=1, **BIGK)
    b, sb = oracle.lpa(g, one_scan=0, **BIGK)
    assert np.array_equal(a, b) and sa == sb
    with pytest.raises(ValueError):
        oracle.louvain(g, one_scan=1)


def test_small_table_hand_trace():
    # Appendix A.2, 3 slots: keys 4, 7, 1 share slot 1 (first key 4), key 5 has slot 2.
    # Vertex 0 sees 4 (w 2), 7 (w 2), 5 (w 3), 1 (w 2): the table holds 4 -> 6 and
    # 5 -> 3, so LPA takes 4; the exact table has 5 as the heaviest single label.
    g, C = _star([2, 2, 3, 2], [4, 7, 5, 1])
    small, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_SMALL, k=3)
    exact, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_EXACT)
    assert small[0] == 4 and exact[0] == 5
    # Louvain reads K_{0->d} from d's slot: with C[0] = 10 (slot 1) the current
    # community already "holds" 6, so no move has a positive gain
    C2 = C.copy()
    C2[0] = 10
    Cn, gain = oracle.move_sweep(g, oracle.ALGO_MOVE, C2, mode=oracle.MODE_SMALL, k=3)
    W = int(np.asarray(g.weights).sum())
    K0 = 9
    Sig = np.bincount(C2, weights=oracle.weighted_degree(g), minlength=g.n)
    # candidate 4 (slot 1, value 6): G = W (6 - 6) - K0 (K0 + Sig[4] - Sig[10])
    g4 = W * 0 - K0 * (K0 + int(Sig[4]) - int(Sig[10]))
    g5 = W * (3 - 6) - K0 * (K0 + int(Sig[5]) - int(Sig[10]))
    assert max(g4, g5) <= 0 and Cn[0] == 10 and gain[0] == 0


def test_small_table_one_slot_takes_first_neighbour():
    # one slot: every key collides; the slot keeps the row's first (non-self) key
    rng = np.random.default_rng(5)
    g = synth.random_small(70, 0.1, 4, seed=5, loops=True)
    C = rng.integers(0, 30, size=g.n).astype(np.int32)
    Cn, _ = oracle.move_sweep(g, oracle.ALGO_LPA, C, mode=oracle.MODE_SMALL, k=1)
    for i in range(g.n):
        nb = [int(j) for j in g.indices[g.offsets[i]:g.offsets[i + 1]] if j != i]
        assert Cn[i] == (C[nb[0]] if nb else C[i])


def test_small_table_without_collisions_is_exact():
    # more slots than labels: no two keys collide and the table is the exact one
    g = synth.random_small(90, 0.15, 5, seed=8)
    for fn in (oracle.lpa, oracle.louvain, oracle.leiden):
        a, sa = fn(g, mode=oracle.MODE_SMALL, k=1 << 20)
        b, sb = fn(g, mode=oracle.MODE_EXACT)
        assert np.array_equal(a, b) and sa == sb


def test_lpa_planted_finds_structure():
    g, truth = synth.planted_exact()
    for mode in (oracle.MODE_EXACT, oracle.MODE_ALG1):
        lab, st = oracle.lpa(g, mode=mode)
        assert st.iterations <= 20
        assert oracle.modularity(g, lab) > 0.6


# ---------------------------------------------------------------------------------
# Louvain
# ---------------------------------------------------------------------------------

def _gold_path3():
    rows = [l.strip() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    sweeps = [r for r in rows if r.startswith("sweep")]
    final = [r for r in rows if r.startswith("final")][0]
    return sweeps, final


@pytest.mark.parametrize("mode", [oracle.MODE_EXACT, oracle.MODE_ALG1])
def test_louvain_path3_trace(mode):
    g = synth.from_edges(3, [(0, 1), (1, 2)])
    sweeps, final = _gold_path3()
    C = np.array([0, 1, 2], np.int32)
    for t, row in enumerate(sweeps):
        _, labs, q = [x.strip() for x in row.split("|")]
        C, _ = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=mode, direction=-1 if t % 2 == 0 else 1)
        assert list(C) == [int(x) for x in labs.split()]
        assert abs(oracle.modularity(g, C) - float(q)) < 1e-12
    parts = [x.strip() for x in final.split("|")]
    lab, st = oracle.louvain(g, mode=mode)
    assert list(lab) == [int(x) for x in parts[1].split()]
    assert st.iterations == int(parts[3].split()[1]) and st.passes == int(parts[4].split()[1])


def _brute_opt(g):
    best = -1.0
    for parts in set_partitions(list(range(g.n))):
        best = max(best, nx_modularity(g, partition_labels(g.n, parts)))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_louvain_not_above_optimum(seed):
    g = synth.random_small(7, 0.45, 4, seed=400 + seed)
    if g.nnz == 0:
        return
    opt = _brute_opt(g)
    for algo in (oracle.louvain, oracle.leiden):
        lab, _ = algo(g, mode=oracle.MODE_EXACT)
        assert oracle.modularity(g, lab) <= opt + 1e-12


def test_louvain_finds_optimum_on_clear_structure():
    edges = clique_edges(range(4)) + clique_edges(range(4, 8)) + [(3, 4)]
    g = synth.from_edges(8, edges)
    opt = _brute_opt(g)
    for algo in (oracle.louvain, oracle.leiden):
        for mode in (oracle.MODE_EXACT, oracle.MODE_ALG1):
            lab, _ = algo(g, mode=mode)
            assert abs(oracle.modularity(g, lab) - opt) < 1e-12
            assert list(lab) == [0] * 4 + [1] * 4
    cl = disjoint_cliques(3, 4)
    for algo in (oracle.louvain, oracle.leiden):
        lab, _ = algo(cl, mode=oracle.MODE_ALG1)
        assert abs(oracle.modularity(cl, lab) - 2 / 3) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_mg_equals_exact_when_k_covers_every_key(seed):
    # No row or aggregation stream has more than 1024 distinct keys, so the sketch
    # never subtracts and MG mode must reproduce exact mode bit for bit.
    g = synth.random_small(60, 0.15, 6, seed=500 + seed)
    for algo in (oracle.lpa, oracle.louvain, oracle.leiden):
        a, sa = algo(g, mode=oracle.MODE_EXACT)
        b, sb = algo(g, mode=oracle.MODE_ALG1, chunk_len=7, **BIGK)
        assert np.array_equal(a, b)
        assert sa.iterations == sb.iterations


def test_thread_count_does_not_matter():
    g = synth.rmat(scale=11, edge_factor=8, seed=11)
    for algo in (oracle.lpa, oracle.louvain, oracle.leiden):
        a, _ = algo(g, threads=1)
        b, _ = algo(g, threads=4)
        assert np.array_equal(a, b)


def test_canonical_labels():
    C = np.array([5, 5, 2, 9, 2, 5], np.int32)
    assert list(oracle.canonical(C)) == [0, 0, 1, 2, 1, 0]


# ---------------------------------------------------------------------------------
# aggregation
# ---------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_exact_aggregation_preserves_modularity(seed):
    rng = np.random.default_rng(600 + seed)
    g = synth.random_small(40, 0.2, 5, seed=600 + seed)
    C = rng.integers(0, 9, size=g.n)
    u, D = np.unique(C, return_inverse=True)
    m = len(u)
    a = oracle.aggregate(g, D.astype(np.int32), m, mode=oracle.MODE_EXACT)
    # the aggregate's row sums are the members' weighted degrees
    K = oracle.weighted_degree(g)
    Ka = oracle.weighted_degree(a)
    assert np.array_equal(Ka, np.bincount(D, weights=K, minlength=m).astype(np.int64))
    # rows sorted, symmetric
    dense = np.zeros((m, m), np.int64)
    for s in range(m):
        row = a.indices[a.offsets[s]:a.offsets[s + 1]]
        assert np.all(np.diff(row) > 0)
        dense[s, row] = a.weights[a.offsets[s]:a.offsets[s + 1]]
    assert np.array_equal(dense, dense.T)
    # modularity of the flattened partition equals that of singletons on the aggregate
    q0 = nx_modularity(g, D)
    q1 = oracle.modularity(a, np.arange(m, dtype=np.int32))
    assert abs(q0 - q1) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_mg_aggregation_bounds(seed):
    rng = np.random.default_rng(700 + seed)
    g = synth.random_small(50, 0.25, 5, seed=700 + seed)
    C = rng.integers(0, 10, size=g.n)
    u, D = np.unique(C, return_inverse=True)
    m = len(u)
    ex = oracle.aggregate(g, D.astype(np.int32), m, mode=oracle.MODE_EXACT)
    exd = {}
    for s in range(m):
        for e in range(ex.offsets[s], ex.offsets[s + 1]):
            exd[(s, int(ex.indices[e]))] = int(ex.weights[e])
    for k in (1, 2, 4):
        for sym in (False, True):
            a = oracle.aggregate(g, D.astype(np.int32), m, mode=oracle.MODE_ALG1, k=k,
                                 chunk_len=9, symmetric=sym)
            seen = {}
            for s in range(m):
                row = a.indices[a.offsets[s]:a.offsets[s + 1]]
                assert np.all(np.diff(row) > 0)
                if not sym:
                    assert len(row) <= k
                for e in range(a.offsets[s], a.offsets[s + 1]):
                    t, v = int(a.indices[e]), int(a.weights[e])
                    assert 0 < v <= exd[(s, t)]
                    seen[(s, t)] = v
            if sym:
                for (s, t), v in seen.items():
                    assert seen[(t, s)] == v


# ---------------------------------------------------------------------------------
# Leiden refinement
# ---------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mode", [oracle.MODE_EXACT, oracle.MODE_ALG1])
def test_refinement_invariants(seed, mode):
    rng = np.random.default_rng(800 + seed)
    g = synth.random_small(60, 0.12, 5, seed=800 + seed)
    bound = rng.integers(0, 4, size=g.n).astype(np.int32)
    R = oracle.refine(g, bound, mode=mode, k=2)
    adj = [set(g.indices[g.offsets[i]:g.offsets[i + 1]].tolist()) for i in range(g.n)]
    for i in range(g.n):
        c = int(R[i])
        assert bound[c] == bound[i]          # inside the bound
        if c != i:
            assert R[c] == c                  # the centre stays
            assert c in adj[i]                # joined along an edge: a star


def test_refinement_mutual_pair():
    # Two vertices joined only to each other propose each other; the higher id
    # joins the lower one.
    g = synth.from_edges(2, [(0, 1)])
    assert list(oracle.refine(g, np.zeros(2, np.int32), mode=oracle.MODE_EXACT)) == [0, 0]
