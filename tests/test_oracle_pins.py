"""Pins for the oracle's refinement scoring, Leiden symmetrisation, aggregation stream
order, Leiden next-pass start and the pass stopping rule (Sections 3.2-3.4, 4.1 Fig. 3,
4.2).  Each expected value comes from something other than the oracle's own formula:
Eq. 1 evaluated exactly (rational arithmetic) on whole partitions, community streams
rebuilt here and folded by the separately pinned sketch, and drivers recomposed here
from separately pinned phases.  Every test also checks that its input is one where the
rule decides the result (a sensitivity witness), so a wrong rule cannot pass by luck."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2411_02268_amd import synth
from _graphs import nx_modularity


# ---------------------------------------------------------------------------------
# Eq. 1 in exact arithmetic (Section 3.2): Q = sum_c [sigma_c / 2m - (Sigma_c / 2m)^2],
# sigma_c the weight of the ordered entries i->j with both ends in c (a self-loop entry
# once), Sigma_c the summed weighted degree of c's members, 2m the sum of all entries.
# ---------------------------------------------------------------------------------

def q_exact(g, C):
    W = int(np.asarray(g.weights, dtype=np.int64).sum())
    sig, tot = {}, {}
    for i in range(g.n):
        ci = int(C[i])
        for e in range(g.offsets[i], g.offsets[i + 1]):
            w = int(g.weights[e])
            tot[ci] = tot.get(ci, 0) + w
            if int(C[g.indices[e]]) == ci:
                sig[ci] = sig.get(ci, 0) + w
    return sum(Fraction(sig.get(c, 0), W) - Fraction(t, W) ** 2 for c, t in tot.items())


def test_q_exact_agrees_with_networkx():
    # the rational Eq. 1 above against the library's modularity (no self-loops)
    for seed in range(4):
        g = synth.random_small(25, 0.25, 5, seed=40 + seed)
        C = np.random.default_rng(seed).integers(0, 5, size=g.n)
        assert abs(float(q_exact(g, C)) - nx_modularity(g, C)) < 1e-12


def neighbours(g, i):
    return [int(j) for j in g.indices[g.offsets[i]:g.offsets[i + 1]]]


# ---------------------------------------------------------------------------------
# Refinement (Section 4.2, Section 3.4): sub-communities start as singletons; a vertex
# scores every neighbour sub-community inside its bound by the modularity change of
# moving there, the change being measured on whole partitions by Eq. 1.
# ---------------------------------------------------------------------------------

def refine_proposals_by_eq1(g, bound):
    """Best target of every vertex, from singleton sub-communities: the neighbour t
    (t != i, same bound) whose joining raises Q the most (> 0; ties to the lowest t)."""
    single = np.arange(g.n)
    q0 = q_exact(g, single)
    prop = np.arange(g.n)
    for i in range(g.n):
        best, bestdq = i, Fraction(0)
        for t in sorted(set(neighbours(g, i))):
            if t == i or bound[t] != bound[i]:
                continue
            C = single.copy()
            C[i] = t
            dq = q_exact(g, C) - q0
            if dq > bestdq:
                best, bestdq = t, dq
        prop[i] = best
    return prop


def accept(prop):
    """Reading of "merges only if no other vertex has joined it" (Section 4.2): i's
    proposal to t stands unless someone other than t proposed i, or t proposed i and
    t > i (the mutual pair joins the lower id)."""
    n = len(prop)
    by = [[] for _ in range(n)]
    for v in range(n):
        if prop[v] != v:
            by[prop[v]].append(v)
    R = np.arange(n)
    for i in range(n):
        t = prop[i]
        if t == i:
            continue
        if not by[i] or (by[i] == [t] and t < i):
            R[i] = t
    return R


def _refine_case(seed):
    rng = np.random.default_rng(900 + seed)
    g = synth.random_small(40, 0.15, 7, seed=900 + seed)
    bound = rng.integers(0, 3, size=g.n).astype(np.int32)
    return g, bound


@pytest.mark.parametrize("seed", range(6))
def test_refinement_scores_targets_by_eq1(seed):
    g, bound = _refine_case(seed)
    prop = refine_proposals_by_eq1(g, bound)
    R = oracle.refine(g, bound, mode=oracle.MODE_EXACT)
    assert np.array_equal(R, accept(prop))
    # MG mode with more slots than any row has keys keeps every candidate
    Rm = oracle.refine(g, bound, mode=oracle.MODE_ALG1, k=64, chunk_len=1 << 40)
    assert np.array_equal(Rm, R)


def test_refinement_target_degree_decides():
    # witness: vertex 0 links with weight 3 to a heavy vertex 1 (K_1 = 3 + 20) and
    # with weight 2 to a light vertex 2 (K_2 = 2).  By Eq. 1 the light target gains
    # more: scoring that ignored the target sub-community's total would pick 1.
    g = synth.from_edges(5, [(0, 1), (0, 2), (1, 3), (1, 4), (3, 4)], [3, 2, 10, 10, 1])
    bound = np.zeros(5, np.int32)
    C1, C2 = np.arange(5), np.arange(5)
    C1[0], C2[0] = 1, 2
    q0 = q_exact(g, np.arange(5))
    assert q_exact(g, C2) - q0 > q_exact(g, C1) - q0 > 0
    prop = refine_proposals_by_eq1(g, bound)
    assert prop[0] == 2
    R = oracle.refine(g, bound, mode=oracle.MODE_EXACT)
    assert np.array_equal(R, accept(prop))


def test_refinement_witness_exists():
    # on the seeds above, scoring without the target's total changes some proposal
    changed = 0
    for seed in range(6):
        g, bound = _refine_case(seed)
        K = oracle.weighted_degree(g)
        W = int(K.sum())
        prop = refine_proposals_by_eq1(g, bound)
        for i in range(g.n):
            cand = {}
            for e in range(g.offsets[i], g.offsets[i + 1]):
                t = int(g.indices[e])
                if t != i and bound[t] == bound[i]:
                    cand[t] = cand.get(t, 0) + int(g.weights[e])
            # a scorer that sees every target with zero total: W*K_it - K_i*K_i
            alt, best = i, 0
            for t in sorted(cand):
                v = W * cand[t] - int(K[i]) * int(K[i])
                if v > best:
                    alt, best = t, v
            changed += alt != prop[i]
    assert changed > 0


# ---------------------------------------------------------------------------------
# Aggregation (Section 4.1 Fig. 3; Section 4.2): community c's stream is its members'
# rows, members in ascending vertex id, each row in CSR order, self-loops kept, key =
# the neighbour's community; the new row is the stream's sketch.  Leiden makes the
# rows symmetric: the union of the kept pairs, weight the larger of the two values.
# ---------------------------------------------------------------------------------

def community_stream(g, D, c, members_order=1):
    mem = [i for i in range(g.n) if D[i] == c][::members_order]
    keys, ws = [], []
    for i in mem:
        for e in range(g.offsets[i], g.offsets[i + 1]):
            keys.append(int(D[g.indices[e]]))
            ws.append(int(g.weights[e]))
    return keys, ws


def rows_from_sketches(g, D, m, k, L, members_order=1):
    return [oracle.sketch_stream(*community_stream(g, D, c, members_order), k=k, chunk_len=L)
            for c in range(m)]


def symmetrise(rows):
    out = [dict() for _ in rows]
    for s, row in enumerate(rows):
        for t, v in row.items():
            out[s][t] = max(out[s].get(t, 0), v)
            out[t][s] = max(out[t].get(s, 0), v)
    return out


def as_rows(a, m):
    return [{int(a.indices[e]): int(a.weights[e]) for e in range(a.offsets[s], a.offsets[s + 1])}
            for s in range(m)]


def _agg_case(seed):
    rng = np.random.default_rng(1000 + seed)
    g = synth.random_small(60, 0.2, 6, seed=1000 + seed, loops=True)
    C = rng.integers(0, 8, size=g.n)
    _, D = np.unique(C, return_inverse=True)
    return g, D.astype(np.int32), int(D.max()) + 1


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("k,L", [(1, 1 << 40), (2, 1 << 40), (3, 7), (2, 5)])
def test_aggregation_rows_are_the_community_stream_sketches(seed, k, L):
    g, D, m = _agg_case(seed)
    want = rows_from_sketches(g, D, m, k, L)
    got = oracle.aggregate(g, D, m, mode=oracle.MODE_ALG1, k=k, chunk_len=L)
    assert as_rows(got, m) == want
    for s in range(m):  # rows ascending by key
        assert np.all(np.diff(got.indices[got.offsets[s]:got.offsets[s + 1]]) > 0)
    sym = oracle.aggregate(g, D, m, mode=oracle.MODE_ALG1, k=k, chunk_len=L, symmetric=True)
    assert as_rows(sym, m) == symmetrise(want)


def test_aggregation_witnesses():
    # the inputs above are ones where member order changes some row, and where some
    # kept pair has different values in its two directions (so min and max differ)
    order_matters = asym = 0
    for seed in range(5):
        g, D, m = _agg_case(seed)
        for k, L in ((2, 1 << 40), (3, 7)):
            fwd = rows_from_sketches(g, D, m, k, L)
            rev = rows_from_sketches(g, D, m, k, L, members_order=-1)
            order_matters += fwd != rev
            for s, row in enumerate(fwd):
                for t, v in row.items():
                    if t != s and s in fwd[t] and fwd[t][s] != v:
                        asym += 1
    assert order_matters > 0 and asym > 0


# ---------------------------------------------------------------------------------
# Drivers recomposed from the pinned phases (Section 3.3 passes; Section 3.4 Leiden):
# local moving (pinned sweeps), refinement (pinned above), aggregation (pinned above),
# dense renumbering in ascending old id.  Leiden's next pass aggregates the refined
# partition and starts every super-vertex in its bound community (Traag et al. 2019).
# ---------------------------------------------------------------------------------

def local_moving(g, C, K, W, tol, mode, k, L, max_it=20):
    it = 0
    for t in range(max_it):
        Sig = np.bincount(C, weights=K, minlength=g.n).astype(np.int64)
        prop, gain = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=mode, k=k, chunk_len=L,
                                       K=K, Sigma=Sig, W=W, direction=0)
        it += 1
        moving = prop != C
        if not moving.any():
            break
        applied, _ = oracle.move_sweep(g, oracle.ALGO_MOVE, C, mode=mode, k=k, chunk_len=L,
                                       K=K, Sigma=Sig, W=W, direction=-1 if t % 2 == 0 else 1)
        dq = Fraction(2 * int(gain[moving].sum()), W * W)  # gain = dQ * W^2 / 2
        C = applied
        if dq <= Fraction(tol).limit_denominator(10**12):
            break
    return C, it


def dense(C):
    _, D = np.unique(C, return_inverse=True)
    return D.astype(np.int32), int(D.max()) + 1 if len(C) else 0


def leiden_recomposed(g0, passes, mode, k, L, tol=1e-2, start_in_bound=True):
    K = oracle.weighted_degree(g0)
    W = int(K.sum())
    g, top = g0, np.arange(g0.n)
    C = np.arange(g.n, dtype=np.int32)
    its = 0
    for p in range(passes):
        C, it = local_moving(g, C, K, W, tol, mode, k, L)
        its += it
        R = oracle.refine(g, C, mode=mode, k=k, chunk_len=L, K=K, W=W)
        D, m = dense(R)
        if p == passes - 1 or m > 0.8 * g.n:
            top = C[top]
            break
        Cd, _ = dense(C)
        top = D[top]
        a = oracle.aggregate(g, D, m, mode=mode, k=k, chunk_len=L, symmetric=True)
        g = synth.CSR(a.offsets, a.indices, a.weights)
        K2 = np.bincount(D, weights=K, minlength=m).astype(np.int64)
        C2 = np.zeros(m, np.int32)
        C2[D] = Cd if start_in_bound else D
        C = C2 if start_in_bound else np.arange(m, dtype=np.int32)
        K = K2
        tol /= 10
    return oracle.canonical(top), its


def louvain_recomposed(g0, passes, mode, k, L, tol=1e-2, agg=None, kagg=None):
    """agg / kagg: the aggregation's mode and slots when they differ from moving's."""
    agg = mode if agg is None else agg
    kagg = k if kagg is None else kagg
    K = oracle.weighted_degree(g0)
    W = int(K.sum())
    g, top = g0, np.arange(g0.n)
    its = 0
    for p in range(passes):
        C, it = local_moving(g, np.arange(g.n, dtype=np.int32), K, W, tol, mode, k, L)
        its += it
        D, m = dense(C)
        top = D[top]
        if p == passes - 1 or m > 0.8 * g.n:
            break
        a = oracle.aggregate(g, D, m, mode=agg, k=kagg, chunk_len=L)
        g = synth.CSR(a.offsets, a.indices, a.weights)
        K = np.bincount(D, weights=K, minlength=m).astype(np.int64)
        tol /= 10
    return oracle.canonical(top), its


def _driver_case(seed):
    return synth.random_small(90, 0.06, 5, seed=1100 + seed)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mode,k,L", [(oracle.MODE_EXACT, 8, 128), (oracle.MODE_ALG1, 2, 5)])
def test_leiden_equals_recomposed_phases(seed, mode, k, L):
    g = _driver_case(seed)
    for passes in (2, 3, 10):
        want, its = leiden_recomposed(g, passes, mode, k, L)
        got, st = oracle.leiden(g, mode=mode, k=k, chunk_len=L, max_passes=passes)
        assert np.array_equal(got, want) and st.iterations == its


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mode,k,L", [(oracle.MODE_EXACT, 8, 128), (oracle.MODE_ALG1, 2, 5)])
def test_louvain_equals_recomposed_phases(seed, mode, k, L):
    g = _driver_case(seed)
    for passes in (2, 10):
        want, its = louvain_recomposed(g, passes, mode, k, L)
        got, st = oracle.louvain(g, mode=mode, k=k, chunk_len=L, max_passes=passes)
        assert np.array_equal(got, want) and st.iterations == its


@pytest.mark.parametrize("seed", range(3))
def test_louvain_aggregation_decoupled_from_moving(seed):
    # aggregation = 1: sketch moving, exact rows; aggregation = 2: exact moving, rows
    # from Algorithm 1 with k_aggregate slots (the measurement of each phase's loss)
    g = _driver_case(seed)
    want, its = louvain_recomposed(g, 10, oracle.MODE_ALG1, 2, 5, agg=oracle.MODE_EXACT)
    got, st = oracle.louvain(g, mode=oracle.MODE_ALG1, k=2, chunk_len=5, aggregation=1)
    assert np.array_equal(got, want) and st.iterations == its
    want, its = louvain_recomposed(g, 10, oracle.MODE_EXACT, 8, 5, agg=oracle.MODE_ALG1, kagg=2)
    got, st = oracle.louvain(g, mode=oracle.MODE_EXACT, k=8, k_aggregate=2, chunk_len=5,
                             aggregation=2)
    assert np.array_equal(got, want) and st.iterations == its
    # the split is not vacuous on these inputs
    full, _ = oracle.louvain(g, mode=oracle.MODE_ALG1, k=2, chunk_len=5)
    ex, _ = oracle.louvain(g, mode=oracle.MODE_EXACT)
    assert not (np.array_equal(full, got) and np.array_equal(ex, got))


def test_leiden_start_witness():
    # on the inputs above, starting the second pass from singletons instead of the
    # bound communities gives different labels for some case
    differ = 0
    for seed in range(4):
        g = _driver_case(seed)
        for mode, k, L in ((oracle.MODE_EXACT, 8, 128), (oracle.MODE_ALG1, 2, 5)):
            a, _ = leiden_recomposed(g, 2, mode, k, L)
            b, _ = leiden_recomposed(g, 2, mode, k, L, start_in_bound=False)
            differ += not np.array_equal(a, b)
    assert differ > 0


# ---------------------------------------------------------------------------------
# Pass stopping rule (Section 3.3): a pass's local moving ends once the modularity
# gained by a sweep's proposed moves, summed, is at most the tolerance.  The gains are
# measured here by Eq. 1 on whole partitions, independently of the oracle's integers.
# ---------------------------------------------------------------------------------

def first_sweep_total_dq(g):
    """Sum over vertices of the best single-vertex modularity gain (> 0) from the
    singleton partition, each gain measured as Q(after) - Q(before) by Eq. 1."""
    C0 = np.arange(g.n)
    q0 = q_exact(g, C0)
    total = Fraction(0)
    for i in range(g.n):
        best = Fraction(0)
        for c in set(neighbours(g, i)) - {i}:
            C = C0.copy()
            C[i] = c
            best = max(best, q_exact(g, C) - q0)
        total += best
    return total


@pytest.mark.parametrize("seed", range(3))
def test_pass_stops_at_tolerance_measured_by_eq1(seed):
    g = synth.random_small(30, 0.2, 5, seed=1200 + seed)
    dq = first_sweep_total_dq(g)
    assert dq > 0
    # just above the first sweep's total gain: one sweep, then stop
    _, st = oracle.louvain(g, mode=oracle.MODE_EXACT, max_passes=1, tolerance=float(dq) * 1.1)
    assert st.iterations == 1
    # just below it: the pass goes on (the second sweep still has moves here)
    _, st = oracle.louvain(g, mode=oracle.MODE_EXACT, max_passes=1, tolerance=float(dq) * 0.9)
    assert st.iterations >= 2
