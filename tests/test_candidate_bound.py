"""The rule by which the Louvain/Leiden decision skips candidates' totals.

The gain of moving vertex i from community d to candidate c (Section 3.2, Eq. 2, in the
integer form the kernels use) is W (k_c - k_d) - K_i (K_i + Sigma_c - Sigma_d).  With
Sigma_c >= 0 it is at most W (k_c - k_d) + K_i (Sigma_d - K_i), which needs no read of
Sigma_c.  The decision scores the heaviest candidate first and then reads another
candidate's total only when that bound can beat the best so far or tie it with a lower
id.  These host-side checks model both decisions over random slots (small ranges, so
that ties and zero gains are frequent) and require them to agree: the pruned decision
is the argmax over all slots with positive gain, lowest id on ties.  The kernels that
implement the rule are compared with the oracle by the GPU parity tests.
"""
import random

EMPTY = -1


def gain(W, kc, kd, Ki, sc, Sd):
    return W * (kc - kd) - Ki * (Ki + sc - Sd)


def better(G, c, best, bestG):
    return best < 0 or G > bestG or (G == bestG and c < best)


def decide_all(W, d, Ki, Sd, kd, keys, ex, sig):
    """Every present candidate other than d scored."""
    best, bestG = -1, 0
    for c, kc in zip(keys, ex):
        if c == EMPTY or c == d:
            continue
        G = gain(W, kc, kd, Ki, sig[c], Sd)
        if G > 0 and better(G, c, best, bestG):
            best, bestG = c, G
    return best, bestG


def decide_pruned(W, d, Ki, Sd, kd, keys, ex, sig):
    """The heaviest candidate first (ties: first slot), then a total read only where
    the bound allows a win or a lower-id tie.  Returns the decision and the reads."""
    best, bestG = -1, 0
    c0, x0 = EMPTY, 0
    for c, kc in zip(keys, ex):
        if c != EMPTY and c != d and (c0 == EMPTY or kc > x0):
            c0, x0 = c, kc
    reads = 0
    if c0 != EMPTY:
        reads += 1
        G = gain(W, x0, kd, Ki, sig[c0], Sd)
        if G > 0:
            best, bestG = c0, G
    live = []
    for c, kc in zip(keys, ex):
        U = W * (kc - kd) + Ki * (Sd - Ki)
        live.append(c != EMPTY and c != d and c != c0 and U > 0 and
                    (best < 0 or U > bestG or (U == bestG and c < best)))
    for (c, kc), lv in zip(zip(keys, ex), live):
        if not lv:
            continue
        reads += 1
        G = gain(W, kc, kd, Ki, sig[c], Sd)
        if G > 0 and better(G, c, best, bestG):
            best, bestG = c, G
    return (best, bestG), reads


def _case(rng, K):
    ncomm = rng.randint(2, 12)
    sig = [rng.randint(0, 6) for _ in range(ncomm)]
    d = rng.randrange(ncomm)
    Ki = rng.randint(0, 4)
    sig[d] = max(sig[d], Ki)  # i belongs to d: Sigma_d >= K_i
    W = rng.randint(1, 8)
    kd = rng.randint(0, 5)
    present = rng.sample(range(ncomm), k=min(ncomm, rng.randint(0, K)))
    keys = present + [EMPTY] * (K - len(present))
    rng.shuffle(keys)
    ex = [rng.randint(0, 6) if c != EMPTY else 0 for c in keys]
    return W, d, Ki, sig[d], kd, keys, ex, sig


def test_pruned_decision_equals_scoring_every_slot():
    rng = random.Random(20241103)
    for K in (1, 2, 4, 8, 16):
        for _ in range(4000):
            W, d, Ki, Sd, kd, keys, ex, sig = _case(rng, K)
            (pb, pg), _ = decide_pruned(W, d, Ki, Sd, kd, keys, ex, sig)
            assert (pb, pg) == decide_all(W, d, Ki, Sd, kd, keys, ex, sig), (W, d, Ki, Sd, kd, keys, ex, sig)


def test_ties_keep_the_lowest_id():
    # two candidates with equal linking weight and equal totals: equal gains, so the
    # lower id must win even though the higher id is the first slot
    W, d, Ki, kd = 4, 0, 1, 0
    sig = [1, 2, 2]
    keys, ex = [2, 1], [3, 3]
    (best, _), _ = decide_pruned(W, d, Ki, sig[d], kd, keys, ex, sig)
    assert best == 1 == decide_all(W, d, Ki, sig[d], kd, keys, ex, sig)[0]


def test_bound_skips_reads_when_one_candidate_dominates():
    # the heaviest candidate's gain exceeds every other candidate's bound: one read
    W, d, Ki, kd = 100, 0, 2, 0
    sig = [2] + [50] * 8
    keys = list(range(1, 9))
    ex = [9, 1, 1, 1, 1, 1, 1, 1]
    (best, _), reads = decide_pruned(W, d, Ki, sig[d], kd, keys, ex, sig)
    assert best == 1 and reads == 1
    assert best == decide_all(W, d, Ki, sig[d], kd, keys, ex, sig)[0]
