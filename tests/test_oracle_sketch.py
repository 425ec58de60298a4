"""Pins for the oracle's sketch (Appendix A.1, Algorithm 1; Section 3.7 for the
Misra-Gries guarantee; Agarwal et al. 2012 for merging).  Nothing here re-types
the oracle: the checks are hand traces, the textbook algorithm, and the error
bounds the mathematics fixes."""
import os
from collections import Counter

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sketch_traces.txt")
MODES = {"alg1": oracle.MODE_ALG1, "std": oracle.MODE_STD, "uncond": oracle.MODE_UNCOND}


def _traces():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, mode, k, stream, final = [x.strip() for x in line.split("|")]
        pairs = [tuple(int(t) for t in x.split(":")) for x in stream.split()]
        exp = {int(a): int(b) for a, b in (x.split(":") for x in final.split())} if final else {}
        out.append((name + "-" + mode, MODES[mode], int(k), pairs, exp))
    return out


@pytest.mark.parametrize("name,mode,k,pairs,exp", _traces(), ids=[t[0] for t in _traces()])
def test_hand_traces(name, mode, k, pairs, exp):
    keys = [p[0] for p in pairs]
    ws = [p[1] for p in pairs]
    assert oracle.sketch_stream(keys, ws, mode=mode, k=k) == exp


def textbook_mg(stream, k):
    """Misra & Gries (1982) frequent items with k counters, unit increments."""
    T = {}
    for x in stream:
        if x in T:
            T[x] += 1
        elif len(T) < k:
            T[x] = 1
        else:
            for y in list(T):
                T[y] -= 1
                if T[y] == 0:
                    del T[y]
    return T


streams = st.lists(st.integers(0, 6), min_size=0, max_size=40)
wstreams = st.lists(st.tuples(st.integers(0, 6), st.integers(1, 9)), min_size=0, max_size=40)


@settings(max_examples=300, deadline=None)
@given(streams, st.integers(1, 6))
def test_unit_weights_equal_textbook_mg(s, k):
    # With unit weights Algorithm 1 is the textbook algorithm (Section 3.7).
    assert oracle.sketch_stream(s, [1] * len(s), k=k) == textbook_mg(s, k)
    assert oracle.sketch_stream(s, [1] * len(s), mode=oracle.MODE_STD, k=k) == textbook_mg(s, k)


@settings(max_examples=300, deadline=None)
@given(wstreams, st.integers(1, 6), st.sampled_from([oracle.MODE_ALG1, oracle.MODE_UNCOND,
                                                     oracle.MODE_STD]))
def test_invariants_any_weights(s, k, mode):
    keys = [a for a, _ in s]
    ws = [b for _, b in s]
    true = Counter()
    for a, b in s:
        true[a] += b
    est = oracle.sketch_stream(keys, ws, mode=mode, k=k)
    assert len(est) <= k
    assert all(v > 0 for v in est.values())
    for key, v in est.items():            # never overcounts
        assert v <= true[key]
    assert sum(est.values()) <= sum(ws)


@settings(max_examples=300, deadline=None)
@given(wstreams, st.integers(1, 6))
def test_textbook_weighted_bound(s, k):
    # Textbook weighted MG: every estimate is within W/(k+1) of the truth.
    keys = [a for a, _ in s]
    ws = [b for _, b in s]
    W = sum(ws)
    true = Counter()
    for a, b in s:
        true[a] += b
    est = oracle.sketch_stream(keys, ws, mode=oracle.MODE_STD, k=k)
    for key in true:
        assert true[key] - est.get(key, 0) <= W / (k + 1) + 1e-9


@settings(max_examples=300, deadline=None)
@given(streams, st.integers(1, 6))
def test_unit_weight_bound_alg1(s, k):
    W = len(s)
    true = Counter(s)
    est = oracle.sketch_stream(s, [1] * W, k=k)
    for key in true:
        assert true[key] - est.get(key, 0) <= W / (k + 1) + 1e-9


@settings(max_examples=200, deadline=None)
@given(wstreams, st.integers(1, 8))
def test_exact_when_k_covers_all_keys(s, k):
    keys = [a for a, _ in s]
    ws = [b for _, b in s]
    true = Counter()
    for a, b in s:
        true[a] += b
    if len(true) <= k:
        # (the unconditional variant subtracts on every miss, so it is not exact)
        for mode in (oracle.MODE_ALG1, oracle.MODE_STD):
            assert oracle.sketch_stream(keys, ws, mode=mode, k=k) == dict(true)
    assert oracle.sketch_stream(keys, ws, mode=oracle.MODE_EXACT, k=k) == dict(true)


def test_alg1_bound_fails_for_unequal_weights():
    # Algorithm 1 is not the textbook weighted algorithm: hand trace W2 loses a key
    # holding 100 of 101 units, beyond W/(k+1).
    est = oracle.sketch_stream([1, 2], [1, 100], k=1)
    assert est == {}


# ---------------------------------------------------------------------------------
# chunk-then-merge
# ---------------------------------------------------------------------------------

@settings(max_examples=200, deadline=None)
@given(wstreams, st.integers(1, 6))
def test_one_chunk_is_plain_alg1(s, k):
    keys = [a for a, _ in s]
    ws = [b for _, b in s]
    a = oracle.sketch_stream(keys, ws, k=k, chunk_len=max(len(s), 1))
    b = oracle.sketch_stream(keys, ws, k=k)
    assert a == b


@settings(max_examples=300, deadline=None)
@given(streams, st.integers(1, 5), st.integers(1, 9))
def test_chunked_unit_weight_bound(s, k, L):
    # Merged MG summaries keep the single-stream guarantee (Agarwal et al. 2012).
    W = len(s)
    true = Counter(s)
    est = oracle.sketch_stream(s, [1] * W, k=k, chunk_len=L)
    assert len(est) <= k
    for key in true:
        assert est.get(key, 0) <= true[key]
        assert true[key] - est.get(key, 0) <= W / (k + 1) + 1e-9


@settings(max_examples=300, deadline=None)
@given(wstreams, st.integers(1, 5), st.integers(1, 9))
def test_chunked_std_bound_any_weights(s, k, L):
    keys = [a for a, _ in s]
    ws = [b for _, b in s]
    W = sum(ws)
    true = Counter()
    for a, b in s:
        true[a] += b
    est = oracle.sketch_stream(keys, ws, mode=oracle.MODE_STD, k=k, chunk_len=L)
    for key in true:
        assert est.get(key, 0) <= true[key]
        assert true[key] - est.get(key, 0) <= W / (k + 1) + 1e-9


def test_chunk_tree_order():
    # 3 chunks of 2 (k=1): chunk sketches {1:2}, {2:2}, {3:2}; the tree merges the
    # first two (equal counts: subtract the 2nd largest -> empty), then carries {3:2}
    # up and merges it with the empty sketch -> {3:2}.  A right-to-left tree would
    # give {1:2}.
    est = oracle.sketch_stream([1, 1, 2, 2, 3, 3], [1] * 6, k=1, chunk_len=2)
    assert est == {3: 2}


@settings(max_examples=300, deadline=None)
@given(st.dictionaries(st.integers(0, 9), st.integers(1, 20), max_size=5),
       st.dictionaries(st.integers(0, 9), st.integers(1, 20), max_size=5), st.integers(1, 5))
def test_merge_properties(a, b, k):
    a = dict(list(a.items())[:k])
    b = dict(list(b.items())[:k])
    m = oracle.mg_merge(a, b, k)
    total = Counter(a) + Counter(b)
    assert len(m) <= k
    for key, v in m.items():
        assert 0 < v <= total[key]
    if len(total) <= k:
        assert m == dict(total)
    # the merge is symmetric in its arguments
    assert oracle.mg_merge(b, a, k) == m


def boyer_moore(keys):
    """Textbook Boyer-Moore majority vote: one candidate and a counter; the same key
    raises the counter, another key lowers it, a zero counter takes the new key."""
    cand, cnt = None, 0
    for x in keys:
        if cnt == 0:
            cand, cnt = x, 1
        elif x == cand:
            cnt += 1
        else:
            cnt -= 1
    return {cand: cnt} if cnt > 0 else {}


@pytest.mark.parametrize("seed", range(8))
def test_one_slot_unit_weights_is_boyer_moore(seed):
    # Algorithm 1 with k = 1 on unit weights is the Boyer-Moore vote (the weighted BM
    # of Section 4.1 reduces to it), so a key held by more than half of the stream
    # is always the surviving candidate
    rng = np.random.default_rng(seed)
    for n in (1, 2, 7, 30, 101):
        keys = rng.integers(0, 4, size=n).tolist()
        assert oracle.sketch_stream(keys, [1] * n, k=1) == boyer_moore(keys)
        maj = [5] * (n // 2 + 1) + rng.integers(0, 4, size=n - n // 2 - 1).tolist()
        rng.shuffle(maj)
        assert list(oracle.sketch_stream(maj, [1] * n, k=1)) == [5]
